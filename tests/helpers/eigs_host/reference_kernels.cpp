// Reference (plain loop) versions of the kernels and of the SpMM that the
// eigensolver driver calls, with the same signatures, so that the driver in
// csrc/eigs.cpp can be run on the CPU (test infrastructure).  A is a CSR set
// by eigs_host_run; X and Y are host arrays.
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "abi_internal.h"

static std::vector<int64_t> g_rp;
static std::vector<int32_t> g_col;
static std::vector<float> g_val;
static std::string g_err;

static uint64_t mix(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

namespace spmm {
int ts_max_outputs() { return 2048; }
int ts_max_width() { return 512; }
size_t ts_partial_doubles() { return 1; }
hipError_t launch_ts_tn(const float* A, ColLayout LA, int p, const float* B, int64_t ldb, int q, int64_t n, double*,
                        double* C, hipStream_t) {
    if (p < 1 || q < 1 || p * q > 2048 || p > 512 || q > 16) return hipErrorInvalidValue;
    for (int a = 0; a < p; ++a)
        for (int c = 0; c < q; ++c) {
            double s = 0.0;
            for (int64_t i = 0; i < n; ++i) s += (double)A[col_off(LA, a) + i * LA.ld] * (double)B[i * ldb + c];
            C[a * q + c] = s;
        }
    return hipSuccess;
}
hipError_t launch_ts_nn(const float* A, ColLayout LA, int p, const double* C, int q, double alpha, double beta,
                        float* W, ColLayout LW, int64_t n, hipStream_t) {
    for (int64_t i = 0; i < n; ++i)
        for (int c = 0; c < q; ++c) {
            double s = 0.0;
            for (int a = 0; a < p; ++a) s += (double)A[col_off(LA, a) + i * LA.ld] * C[a * q + c];
            float* w = W + col_off(LW, c) + i * LW.ld;
            const double old = alpha != 0.0 ? alpha * (double)*w : 0.0;
            *w = (float)(old + beta * s);
        }
    return hipSuccess;
}
hipError_t launch_fill_uniform(float* X, int64_t ldx, int q, int64_t n, uint64_t seed, hipStream_t) {
    for (int64_t i = 0; i < n; ++i)
        for (int c = 0; c < q; ++c)
            X[i * ldx + c] = (float)(mix(seed ^ mix((uint64_t)i * 64u + (uint64_t)c)) >> 40) * (1.0f / 16777216.0f) - 0.5f;
    return hipSuccess;
}
}  // namespace spmm

namespace spmm_abi {
spmm_status_t fail(spmm_status_t st, const std::string& msg) {
    g_err = msg;
    return st;
}
spmm_status_t hip_fail(hipError_t, const char* what) {
    g_err = what;
    return SPMM_EHIP;
}
spmm_status_t prepare_device(spmm::Handle&) { return SPMM_OK; }
spmm_status_t run_device(spmm::Handle& H, const void* Xv, int k, int64_t ldx, int, const float*, float* Y, int64_t ldy,
                         hipStream_t, bool) {
    const float* X = static_cast<const float*>(Xv);
    for (int64_t r = 0; r < H.n_rows; ++r)
        for (int c = 0; c < k; ++c) {
            double s = 0.0;
            for (int64_t e = g_rp[r]; e < g_rp[r + 1]; ++e)
                s += (g_val.empty() ? 1.0 : (double)g_val[e]) * (double)X[(int64_t)g_col[e] * ldx + c];
            Y[r * ldy + c] = (float)s;
        }
    return SPMM_OK;
}
}  // namespace spmm_abi

extern "C" spmm_status_t spmm_stream_run(spmm_handle_t h, const void* X, int k, int64_t ldx, spmm_xdtype_t dt,
                                         const float* cs, float* Y, int64_t ldy, hipStream_t s, hipStream_t) {
    return spmm_abi::run_device(h->H, X, k, ldx, dt, cs, Y, ldy, s, false);
}

// Run spmm_eigs on the CSR (row_ptr, col, val or NULL); info4 receives
// n_converged, restarts, n_spmm, max_dim.
extern "C" int eigs_host_run(int64_t n, const int64_t* rp, const int32_t* col, const float* val, int nev, int block,
                             int max_dim, int which, double tol, int max_restarts, uint64_t seed, double* evals,
                             float* evecs, double* resid, int* info4) {
    g_rp.assign(rp, rp + n + 1);
    g_col.assign(col, col + rp[n]);
    g_val.clear();
    if (val) g_val.assign(val, val + rp[n]);
    spmm_handle_s h;
    h.H.n_rows = n;
    h.H.n_cols = n;
    h.H.place = SPMM_PLACE_DEVICE;
    spmm_eigs_opts o{};
    o.nev = nev;
    o.block = block;
    o.max_dim = max_dim;
    o.which = which;
    o.tol = tol;
    o.max_restarts = max_restarts;
    o.seed = seed;
    spmm_eigs_info inf{};
    const int st = spmm_eigs(&h, &o, evals, evecs, nev, resid, &inf, nullptr);
    info4[0] = inf.n_converged;
    info4[1] = inf.restarts;
    info4[2] = (int)inf.n_spmm;
    info4[3] = inf.max_dim;
    return st;
}

extern "C" const char* eigs_host_error() { return g_err.c_str(); }

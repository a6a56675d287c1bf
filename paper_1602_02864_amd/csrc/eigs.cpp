// Block Krylov-Schur eigensolver for a symmetric sparse matrix on the device
// (the eigensolver application of Section 4.2): the sparse products are the
// library's SpMM, the basis and its dense updates stay in HBM, and only the
// small projected matrices come back to the host.
//
// For a symmetric A the Krylov-Schur method (Stewart, SIAM J. Matrix Anal.
// Appl. 23(3), 2001) is thick-restart block Lanczos: expand an orthonormal
// basis V block by block (W = A V_j, orthogonalised against all of V twice,
// then made orthonormal), keep T = V^T A V, and when V holds m columns take
// the Ritz pairs of T, stop if the wanted ones have small residuals, else
// keep the best p Ritz vectors plus the residual block and expand again.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <numeric>
#include <vector>

#include "abi_internal.h"
#include "spmm.h"

using spmm_abi::fail;
using spmm_abi::hip_fail;

namespace {

// Cyclic Jacobi eigen-decomposition of a symmetric matrix (Golub and Van
// Loan, Matrix Computations, the symmetric Schur decomposition by plane
// rotations).  a: n x n row-major, overwritten.  On return w[j] is an
// eigenvalue and column j of z (n x n row-major) its unit eigenvector;
// unsorted.
void jacobi_eig(int n, std::vector<double>& a, std::vector<double>& w, std::vector<double>& z) {
    z.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) z[(size_t)i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) (i == j ? diag : off) += a[(size_t)i * n + j] * a[(size_t)i * n + j];
        if (off == 0.0 || off <= 1e-30 * diag) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = a[(size_t)p * n + q];
                if (apq == 0.0) continue;
                const double tau = (a[(size_t)q * n + q] - a[(size_t)p * n + p]) / (2.0 * apq);
                const double t = (tau >= 0.0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
                const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
                for (int k = 0; k < n; ++k) {  // columns p, q of a J
                    const double x = a[(size_t)k * n + p], y = a[(size_t)k * n + q];
                    a[(size_t)k * n + p] = c * x - s * y;
                    a[(size_t)k * n + q] = s * x + c * y;
                }
                for (int k = 0; k < n; ++k) {  // rows p, q of J^T (a J)
                    const double x = a[(size_t)p * n + k], y = a[(size_t)q * n + k];
                    a[(size_t)p * n + k] = c * x - s * y;
                    a[(size_t)q * n + k] = s * x + c * y;
                }
                for (int k = 0; k < n; ++k) {
                    const double x = z[(size_t)k * n + p], y = z[(size_t)k * n + q];
                    z[(size_t)k * n + p] = c * x - s * y;
                    z[(size_t)k * n + q] = s * x + c * y;
                }
            }
    }
    w.resize(n);
    for (int i = 0; i < n; ++i) w[i] = a[(size_t)i * n + i];
}

// Indices of w in the order the wanted end of the spectrum comes first.
std::vector<int> ritz_order(const std::vector<double>& w, int which) {
    std::vector<int> o(w.size());
    std::iota(o.begin(), o.end(), 0);
    std::stable_sort(o.begin(), o.end(), [&](int x, int y) {
        if (which == SPMM_EIGS_LA) return w[x] > w[y];
        if (which == SPMM_EIGS_SA) return w[x] < w[y];
        const double ax = std::fabs(w[x]), ay = std::fabs(w[y]);
        return ax != ay ? ax > ay : w[x] > w[y];
    });
    return o;
}

uint64_t mix64(uint64_t z) {  // SplitMix64 finaliser: seeds of successive random blocks
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Directions of a block whose squared singular value is below this fraction
// of the block's squared norm before orthogonalisation are taken as lost to
// rounding (FP32 basis) and replaced by random ones.
constexpr double kRankTol = 1e-12;

struct Solver {
    spmm_handle_t h;
    spmm::Handle& H;
    hipStream_t s;
    hipStream_t copy = nullptr;  // tiles in host memory: the stream of the tile copies
    int64_t n;
    int b, m;
    // The basis: for b >= 4, blocks of b columns, each n x b contiguous; for
    // narrower blocks row-major with m + b columns (contiguous blocks of one
    // or two columns would make the basis kernels read one float per line
    // per lane).  Block c / b starts at col_off(VL, c), row stride VL.ld.
    spmm::ColLayout VL;
    float* V[2];
    float* W;
    float* Z;    // n x b scratch block
    double* part;
    double* dC;  // coefficients of one block, (m + b) x b
    double* dM;  // small dense factors, (m + b) x (m + b)
    uint64_t seed;
    uint64_t n_fill = 0;
    int64_t n_spmm = 0;
    int64_t n_first_pass = 0, n_second_pass = 0;   // block projections, and how many needed a second
    double spmm_ms = 0.0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // dense kernels: an event pair around each launch (read back at the end)
    // and the algorithmic HBM bytes of each
    std::vector<hipEvent_t> dense_ev;
    size_t dense_used = 0;
    double dense_bytes = 0.0;

    hipError_t dense_mark() {
        if (dense_used == dense_ev.size()) {
            hipEvent_t e = nullptr;
            hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) return r;
            dense_ev.push_back(e);
        }
        return hipEventRecord(dense_ev[dense_used++], s);
    }
    spmm_status_t dense_ms(double& ms) {
        ms = 0.0;
        for (size_t i = 0; i + 1 < dense_used; i += 2) {
            hipError_t e = hipEventSynchronize(dense_ev[i + 1]);
            float t = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&t, dense_ev[i], dense_ev[i + 1]);
            if (e != hipSuccess) return hip_fail(e, "dense kernel timing");
            ms += t;
        }
        return SPMM_OK;
    }

    spmm_status_t sync(const char* what) {
        hipError_t e = hipStreamSynchronize(s);
        return e == hipSuccess ? SPMM_OK : hip_fail(e, what);
    }
    spmm_status_t get(double* host, const double* dev, size_t count) {
        hipError_t e = hipMemcpyAsync(host, dev, count * sizeof(double), hipMemcpyDeviceToHost, s);
        return e == hipSuccess ? SPMM_OK : hip_fail(e, "copy to host");
    }
    spmm_status_t put(double* dev, const double* host, size_t count) {
        hipError_t e = hipMemcpyAsync(dev, host, count * sizeof(double), hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "copy to device");
        // the host vector may change right after the call returns
        return sync("copy to device");
    }
    spmm_status_t tn(const float* A, spmm::ColLayout LA, int p, const float* B, int64_t ldb, int q, double* C) {
        hipError_t e = dense_mark();
        if (e == hipSuccess) e = spmm::launch_ts_tn(A, LA, p, B, ldb, q, n, part, C, s);
        if (e == hipSuccess) e = dense_mark();
        dense_bytes += 4.0 * (double)n * (p + q);
        return e == hipSuccess ? SPMM_OK : hip_fail(e, "basis product launch");
    }
    spmm_status_t nn(const float* A, spmm::ColLayout LA, int p, const double* C, int q, double alpha, double beta,
                     float* Wo, spmm::ColLayout LW) {
        hipError_t e = dense_mark();
        if (e == hipSuccess) e = spmm::launch_ts_nn(A, LA, p, C, q, alpha, beta, Wo, LW, n, s);
        if (e == hipSuccess) e = dense_mark();
        dense_bytes += 4.0 * (double)n * (p + (alpha != 0.0 ? 2 : 1) * q);
        return e == hipSuccess ? SPMM_OK : hip_fail(e, "basis update launch");
    }
    spmm_status_t fill(float* X, int64_t ldx, int q) {
        hipError_t e = spmm::launch_fill_uniform(X, ldx, q, n, mix64(seed + ++n_fill), s);
        return e == hipSuccess ? SPMM_OK : hip_fail(e, "random fill launch");
    }

    // Y (n x b, stride b) = A X for a block of b basis columns (stride
    // VL.ld), timed with events.
    spmm_status_t product(const float* X, float* Y) {
        hipError_t e;
        if ((e = hipEventRecord(ev0, s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
        spmm_status_t st = H.place == SPMM_PLACE_DEVICE
                               ? spmm_abi::run_device(H, X, b, VL.ld, SPMM_X_F32, nullptr, Y, b, s, false)
                               : spmm_stream_run(h, X, b, VL.ld, SPMM_X_F32, nullptr, Y, b, s, copy);
        if (st != SPMM_OK) return st;
        if ((e = hipEventRecord(ev1, s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
        if ((e = hipEventSynchronize(ev1)) != hipSuccess) return hip_fail(e, "SpMM");
        float ms = 0.0f;
        if ((e = hipEventElapsedTime(&ms, ev0, ev1)) != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
        spmm_ms += ms;
        ++n_spmm;
        return SPMM_OK;
    }

    // X (n x q, stride ldx) -= Vb Vb^T X twice, Vb = first nb columns of Vc.
    // coef (nb x q) receives the sum of both coefficient blocks; norm2 the
    // squared Frobenius norm of the first one.
    spmm_status_t project_out(const float* Vc, int nb, float* X, int64_t ldx, int q, std::vector<double>& coef,
                              double& norm2) {
        coef.assign((size_t)nb * q, 0.0);
        norm2 = 0.0;
        std::vector<double> c((size_t)nb * q);
        spmm_status_t st;
        for (int pass = 0; pass < 2; ++pass) {
            if ((st = tn(Vc, VL, nb, X, ldx, q, dC)) != SPMM_OK) return st;
            if ((st = nn(Vc, VL, nb, dC, q, 1.0, -1.0, X, spmm::row_major(ldx))) != SPMM_OK) return st;
            if ((st = get(c.data(), dC, c.size())) != SPMM_OK) return st;
            if ((st = sync("projection")) != SPMM_OK) return st;
            for (size_t i = 0; i < c.size(); ++i) {
                coef[i] += c[i];
                if (pass == 0) norm2 += c[i] * c[i];
            }
        }
        return SPMM_OK;
    }

    // Gram matrix G = X^T X (q x q) of a device block, on the host.
    spmm_status_t gram(const float* X, int64_t ldx, int q, std::vector<double>& G) {
        G.resize((size_t)q * q);
        spmm_status_t st = tn(X, spmm::row_major(ldx), q, X, ldx, q, dC);
        if (st == SPMM_OK) st = get(G.data(), dC, G.size());
        if (st == SPMM_OK) st = sync("Gram matrix");
        return st;
    }

    // Dst (n x b, stride ldd) = Src (n x b, stride lds) G^{-1/2} for the Gram
    // matrix G of Src (symmetric inverse square root from G's eigenvectors):
    // one SVQB pass (Stathopoulos and Wu, SIAM J. Sci. Comput. 23(6), 2002).
    // w, U: G's eigen-decomposition if already known, else empty.  sqrtG, if
    // given, receives G^{1/2} (Src = Dst G^{1/2}).
    spmm_status_t svqb(const float* Src, int64_t lds, float* Dst, int64_t ldd, std::vector<double> w = {},
                       std::vector<double> U = {}, std::vector<double>* sqrtG = nullptr) {
        spmm_status_t st;
        if (w.empty()) {
            std::vector<double> G;
            if ((st = gram(Src, lds, b, G)) != SPMM_OK) return st;
            jacobi_eig(b, G, w, U);
        }
        const double wmax = *std::max_element(w.begin(), w.end());
        const double wmin = *std::min_element(w.begin(), w.end());
        if (!(wmax > 0.0) || !(wmin > 1e-10 * wmax)) return fail(SPMM_ENOTCONV, "a basis block lost its rank");
        std::vector<double> M((size_t)b * b, 0.0);
        for (int i = 0; i < b; ++i)
            for (int j = 0; j < b; ++j) {
                double v = 0.0;
                for (int l = 0; l < b; ++l) v += U[(size_t)i * b + l] * U[(size_t)j * b + l] / std::sqrt(w[l]);
                M[(size_t)i * b + j] = v;
            }
        if (sqrtG) {
            sqrtG->assign((size_t)b * b, 0.0);
            for (int i = 0; i < b; ++i)
                for (int j = 0; j < b; ++j) {
                    double v = 0.0;
                    for (int l = 0; l < b; ++l) v += U[(size_t)i * b + l] * U[(size_t)j * b + l] * std::sqrt(w[l]);
                    (*sqrtG)[(size_t)i * b + j] = v;
                }
        }
        if ((st = put(dM, M.data(), M.size())) != SPMM_OK) return st;
        return nn(Src, spmm::row_major(lds), b, dM, b, 0.0, 1.0, Dst, spmm::row_major(ldd));
    }

    // Make the block W (n x b, stride b) orthogonal to the first nb columns
    // of Vc and orthonormal, writing it to the basis block Dst (stride
    // VL.ld): W ~ Dst R.  coef
    // receives Vb^T W (nb x b), R (b x b) is Dst^T W after the projection
    // (from the two Gram matrices when W has full rank).  Directions of W
    // lost to cancellation are replaced by random vectors orthogonal to the
    // basis (a breakdown of the Krylov space), with R = Dst^T W computed
    // explicitly so that the Krylov relation keeps holding.
    spmm_status_t orthonormalise(const float* Vc, int nb, float* Dst, std::vector<double>& coef,
                                 std::vector<double>& R) {
        spmm_status_t st;
        double scale2 = 0.0;
        std::vector<double> G, w, U;
        if (nb > 0) {
            // one projection, and a second one only where the first cancelled
            // a column of W by more than a factor 1/sqrt(2) (Daniel, Gragg,
            // Kaufman and Stewart, Math. Comp. 30, 1976): with FP64 sums the
            // first pass leaves W orthogonal to V to within V's own
            // orthogonality times that factor
            std::vector<double> c1((size_t)nb * b);
            if ((st = tn(Vc, VL, nb, W, b, b, dC)) != SPMM_OK) return st;
            if ((st = nn(Vc, VL, nb, dC, b, 1.0, -1.0, W, spmm::row_major(b))) != SPMM_OK) return st;
            if ((st = get(c1.data(), dC, c1.size())) != SPMM_OK) return st;
            if ((st = gram(W, b, b, G)) != SPMM_OK) return st;
            coef = c1;
            bool again = false;
            for (int c = 0; c < b; ++c) {
                double w0 = G[(size_t)c * b + c];
                for (int r = 0; r < nb; ++r) w0 += c1[(size_t)r * b + c] * c1[(size_t)r * b + c];
                if (G[(size_t)c * b + c] < 0.5 * w0) again = true;
            }
            for (double v : c1) scale2 += v * v;
            if (again) {
                ++n_second_pass;
                if ((st = tn(Vc, VL, nb, W, b, b, dC)) != SPMM_OK) return st;
                if ((st = nn(Vc, VL, nb, dC, b, 1.0, -1.0, W, spmm::row_major(b))) != SPMM_OK) return st;
                if ((st = get(c1.data(), dC, c1.size())) != SPMM_OK) return st;
                if ((st = gram(W, b, b, G)) != SPMM_OK) return st;
                for (size_t i = 0; i < c1.size(); ++i) coef[i] += c1[i];
            }
            ++n_first_pass;
        } else if ((st = gram(W, b, b, G)) != SPMM_OK) {
            return st;
        }
        for (int i = 0; i < b; ++i) scale2 += G[(size_t)i * b + i];
        jacobi_eig(b, G, w, U);
        std::vector<int> keep;
        for (int l = 0; l < b; ++l)
            if (w[l] > kRankTol * scale2 && w[l] > 0.0) keep.push_back(l);
        const int r = (int)keep.size();
        std::vector<double> s1, s2;
        if (r == b) {
            if ((st = svqb(W, b, Z, b, w, U, &s1)) != SPMM_OK) return st;
        } else {
            // Z[:, 0:r] = W U_keep diag(1/sqrt(w_keep)), then random columns
            std::vector<double> M((size_t)b * std::max(r, 1), 0.0);
            for (int i = 0; i < b; ++i)
                for (int j = 0; j < r; ++j)
                    M[(size_t)i * r + j] = U[(size_t)i * b + keep[j]] / std::sqrt(w[keep[j]]);
            if (r > 0) {
                if ((st = put(dM, M.data(), (size_t)b * r)) != SPMM_OK) return st;
                if ((st = nn(W, spmm::row_major(b), b, dM, r, 0.0, 1.0, Z, spmm::row_major(b))) != SPMM_OK)
                    return st;
            }
            if ((st = fill(Z + r, b, b - r)) != SPMM_OK) return st;
            std::vector<double> unused;
            double unused2;
            if (nb > 0 && (st = project_out(Vc, nb, Z, b, b, unused, unused2)) != SPMM_OK) return st;
            if ((st = svqb(Z, b, Dst, VL.ld)) != SPMM_OK) return st;
            hipError_t e = hipMemcpy2DAsync(Z, (size_t)b * sizeof(float), Dst, (size_t)VL.ld * sizeof(float),
                                            (size_t)b * sizeof(float), (size_t)n, hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) return hip_fail(e, "basis block copy");
        }
        // second pass for orthogonality within the block
        if ((st = svqb(Z, b, Dst, VL.ld, {}, {}, &s2)) != SPMM_OK) return st;
        R.resize((size_t)b * b);
        if (r == b) {
            // W = Z G1^{1/2} and Z = Dst G2^{1/2}, so R = G2^{1/2} G1^{1/2}:
            // no pass over the new block
            for (int i = 0; i < b; ++i)
                for (int j = 0; j < b; ++j) {
                    double v = 0.0;
                    for (int l = 0; l < b; ++l) v += s2[(size_t)i * b + l] * s1[(size_t)l * b + j];
                    R[(size_t)i * b + j] = v;
                }
            return SPMM_OK;
        }
        if ((st = tn(Dst, spmm::row_major(VL.ld), b, W, b, b, dC)) != SPMM_OK) return st;
        if ((st = get(R.data(), dC, R.size())) != SPMM_OK) return st;
        return sync("block orthonormalisation");
    }
};

}  // namespace

extern "C" size_t spmm_dense_tn_workspace(int64_t n, int p, int q) {
    (void)n;
    if (p < 1 || q < 1) return 0;
    return spmm::ts_partial_doubles() * sizeof(double);
}

extern "C" spmm_status_t spmm_dense_tn(const float* A, int64_t lda, int p, const float* B, int64_t ldb, int q,
                                       int64_t n, double* C, void* work, size_t work_bytes, hipStream_t s) {
    if (p < 1 || q < 1 || p > spmm::ts_max_width() || q > 16 || p * q > spmm::ts_max_outputs() || n < 0)
        return fail(SPMM_EINVAL, "need 1 <= p <= " + std::to_string(spmm::ts_max_width()) + ", 1 <= q <= 16, p q <= " +
                                     std::to_string(spmm::ts_max_outputs()) + ", n >= 0");
    if (lda < p || ldb < q) return fail(SPMM_EINVAL, "lda must be >= p and ldb >= q");
    if (!C || !work || (n > 0 && (!A || !B))) return fail(SPMM_EINVAL, "NULL argument");
    if (work_bytes < spmm_dense_tn_workspace(n, p, q)) return fail(SPMM_EINVAL, "workspace too small");
    hipError_t e = spmm::launch_ts_tn(A, spmm::row_major(lda), p, B, ldb, q, n, static_cast<double*>(work), C, s);
    return e == hipSuccess ? SPMM_OK : hip_fail(e, "basis product launch");
}

extern "C" spmm_status_t spmm_dense_nn(const float* A, int64_t lda, int p, const double* C, int q, double alpha,
                                       double beta, float* W, int64_t ldw, int64_t n, hipStream_t s) {
    if (p < 1 || q < 1 || n < 0) return fail(SPMM_EINVAL, "need p >= 1, q >= 1, n >= 0");
    if (lda < p || ldw < q) return fail(SPMM_EINVAL, "lda must be >= p and ldw >= q");
    if (n > 0 && (!A || !C || !W)) return fail(SPMM_EINVAL, "NULL argument");
    hipError_t e = spmm::launch_ts_nn(A, spmm::row_major(lda), p, C, q, alpha, beta, W, spmm::row_major(ldw), n, s);
    return e == hipSuccess ? SPMM_OK : hip_fail(e, "basis update launch");
}

extern "C" spmm_status_t spmm_sym_eig_small(int n, const double* a, double* w, double* z) {
    if (n < 1 || n > 1024 || !a || !w || !z) return fail(SPMM_EINVAL, "need 1 <= n <= 1024 and non-NULL arrays");
    std::vector<double> A(a, a + (size_t)n * n), wv, zv;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < i; ++j)
            if (A[(size_t)i * n + j] != A[(size_t)j * n + i]) return fail(SPMM_EINVAL, "matrix is not symmetric");
    jacobi_eig(n, A, wv, zv);
    std::vector<int> o = ritz_order(wv, SPMM_EIGS_SA);
    for (int j = 0; j < n; ++j) {
        w[j] = wv[o[j]];
        for (int i = 0; i < n; ++i) z[(size_t)i * n + j] = zv[(size_t)i * n + o[j]];
    }
    return SPMM_OK;
}

extern "C" spmm_status_t spmm_eigs(spmm_handle_t h, const spmm_eigs_opts* o, double* evals, float* evecs,
                                   int64_t ldvec, double* resid, spmm_eigs_info* info, hipStream_t s) {
    const auto t_start = std::chrono::steady_clock::now();
    try {
        if (!h || !o || !evals) return fail(SPMM_EINVAL, "NULL argument");
        spmm::Handle& H = h->H;
        if (H.n_rows != H.n_cols) return fail(SPMM_EINVAL, "the matrix must be square (and symmetric)");
        const int64_t n = H.n_rows;
        const int nev = o->nev;
        const int b = o->block == 0 ? 4 : o->block;
        if (nev < 1 || b < 1 || b > 16) return fail(SPMM_EINVAL, "need nev >= 1 and block in 1..16");
        if (o->which != SPMM_EIGS_LM && o->which != SPMM_EIGS_LA && o->which != SPMM_EIGS_SA)
            return fail(SPMM_EINVAL, "which must be SPMM_EIGS_LM, _LA or _SA");
        const double tol = o->tol == 0.0 ? 1e-5 : o->tol;
        if (!(tol > 0.0) || o->max_restarts < 0) return fail(SPMM_EINVAL, "need tol > 0 (0 selects 1e-5) and max_restarts >= 0");
        const int max_restarts = o->max_restarts == 0 ? 500 : o->max_restarts;
        int m = o->max_dim;
        if (m == 0) {
            // a wide basis: power-law spectra have clustered top eigenvalues,
            // and restarting a narrow basis converges slowly; a block method
            // needs about 24 blocks for the same polynomial degree
            const int64_t cap = std::min<int64_t>({spmm::ts_max_outputs() / b, spmm::ts_max_width() - b, n - b});
            // (measured on a 67M-vertex graph: b = 8 took 46 products with
            // m = 192 and 37 with m = 128), but no wider than needed
            const int want = std::min(std::max({6 * nev, nev + 4 * b, 24 * b}), std::max(128, 8 * nev + 4 * b));
            m = (int)std::min<int64_t>(((want + b - 1) / b) * b, cap / b * b);
        }
        if (m % b != 0 || m < nev + b) return fail(SPMM_EINVAL, "max_dim must be a multiple of block and >= nev + block");
        if ((int64_t)m + b > n) return fail(SPMM_EINVAL, "max_dim + block exceeds the matrix order");
        if (m * b > spmm::ts_max_outputs() || m + b > spmm::ts_max_width())
            return fail(SPMM_EINVAL, "need max_dim * block <= " + std::to_string(spmm::ts_max_outputs()) +
                                         " and max_dim + block <= " + std::to_string(spmm::ts_max_width()));
        if (evecs && ldvec < nev) return fail(SPMM_EINVAL, "ldvec must be >= nev");
        spmm_status_t st = spmm_abi::prepare_device(H);
        if (st != SPMM_OK) return st;
        hipError_t e;
        // tiles in host memory: the solver runs on streams of its own (the
        // products stream the tiles on a copy stream, as spmm_stream_run)
        // after the work already queued on s
        struct OwnStreams {
            hipStream_t compute = nullptr, copy = nullptr;
            ~OwnStreams() {
                if (compute) (void)hipStreamSynchronize(compute);
                if (copy) (void)hipStreamSynchronize(copy);
                if (compute) (void)hipStreamDestroy(compute);
                if (copy) (void)hipStreamDestroy(copy);
            }
        } own;
        if (H.place != SPMM_PLACE_DEVICE) {
            if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "caller stream");
            if ((e = hipStreamCreateWithFlags(&own.compute, hipStreamNonBlocking)) != hipSuccess ||
                (e = hipStreamCreateWithFlags(&own.copy, hipStreamNonBlocking)) != hipSuccess)
                return hip_fail(e, "hipStreamCreate");
            s = own.compute;
        }

        spmm_abi::DevBufs bufs;
        Solver S{h, H, s, own.copy, n, b, m, b >= 4 ? spmm::ColLayout{b, b, n * b} : spmm::row_major(m + b)};
        S.V[0] = bufs.get<float>((size_t)n * (m + b));
        S.V[1] = bufs.get<float>((size_t)n * (m + b));
        S.W = bufs.get<float>((size_t)n * b);
        S.Z = bufs.get<float>((size_t)n * b);
        S.part = bufs.get<double>(spmm::ts_partial_doubles());
        S.dC = bufs.get<double>((size_t)(m + b) * b);
        S.dM = bufs.get<double>((size_t)(m + b) * (m + b));
        if (!S.V[0] || !S.V[1] || !S.W || !S.Z || !S.part || !S.dC || !S.dM)
            return fail(SPMM_ENOMEM, "hipMalloc(eigensolver workspace) failed");
        S.seed = o->seed;
        struct Cleanup {  // the workspace is freed on return: finish the work that uses it first
            Solver& S;
            ~Cleanup() {
                (void)hipStreamSynchronize(S.s);
                if (S.ev0) (void)hipEventDestroy(S.ev0);
                if (S.ev1) (void)hipEventDestroy(S.ev1);
                for (hipEvent_t e : S.dense_ev) (void)hipEventDestroy(e);
            }
        } cleanup{S};
        if ((e = hipEventCreate(&S.ev0)) != hipSuccess || (e = hipEventCreate(&S.ev1)) != hipSuccess)
            return hip_fail(e, "hipEventCreate");

        int cur_buf = 0;
        float* Vc = S.V[0];
        // starting block: random, orthonormal
        std::vector<double> coef, R, E((size_t)b * b, 0.0);
        if ((st = S.fill(S.W, b, b)) != SPMM_OK) return st;
        if ((st = S.orthonormalise(Vc, 0, Vc, coef, R)) != SPMM_OK) return st;

        const int ldt = m + b;
        std::vector<double> T((size_t)ldt * ldt, 0.0);
        auto t = [&](int r, int c) -> double& { return T[(size_t)r * ldt + c]; };
        int cur = 0, restarts = 0, n_conv = 0;
        std::vector<double> theta, Sv, rnorm;
        std::vector<int> order;
        for (;;) {
            // expand the basis to m columns, one block at a time
            while (cur < m) {
                const int nb = cur + b;
                // the block of basis columns cur .. cur + b - 1 starts at col_off(VL, cur)
                if ((st = S.product(Vc + spmm::col_off(S.VL, cur), S.W)) != SPMM_OK) return st;
                if ((st = S.orthonormalise(Vc, nb, Vc + spmm::col_off(S.VL, nb), coef, R)) != SPMM_OK) return st;
                for (int r = 0; r < nb; ++r)
                    for (int x = 0; x < b; ++x) {
                        const double v = coef[(size_t)r * b + x];
                        if (r < cur) {
                            t(r, cur + x) = v;
                            t(cur + x, r) = v;
                        }
                    }
                for (int x = 0; x < b; ++x)
                    for (int y = 0; y < b; ++y)
                        t(cur + x, cur + y) = 0.5 * (coef[(size_t)(cur + x) * b + y] + coef[(size_t)(cur + y) * b + x]);
                if (nb < m) {
                    for (int x = 0; x < b; ++x)
                        for (int y = 0; y < b; ++y) {
                            t(nb + x, cur + y) = R[(size_t)x * b + y];
                            t(cur + y, nb + x) = R[(size_t)x * b + y];
                        }
                } else {
                    E = R;
                }
                cur = nb;
            }
            // Rayleigh-Ritz on T (m x m)
            std::vector<double> Tm((size_t)m * m);
            for (int r = 0; r < m; ++r)
                for (int c = 0; c < m; ++c) Tm[(size_t)r * m + c] = t(r, c);
            jacobi_eig(m, Tm, theta, Sv);
            order = ritz_order(theta, o->which);
            // residual of Ritz pair i: || E * (last b rows of its eigenvector) ||
            rnorm.assign(m, 0.0);
            for (int i = 0; i < m; ++i) {
                double ss = 0.0;
                for (int x = 0; x < b; ++x) {
                    double v = 0.0;
                    for (int y = 0; y < b; ++y) v += E[(size_t)x * b + y] * Sv[(size_t)(m - b + y) * m + order[i]];
                    ss += v * v;
                }
                rnorm[i] = std::sqrt(ss);
            }
            n_conv = 0;
            for (int i = 0; i < nev; ++i)
                if (rnorm[i] <= tol * std::fabs(theta[order[i]])) ++n_conv;
            if (n_conv == nev || restarts == max_restarts) break;
            // restart: keep p Ritz vectors and the residual block
            const int p_want = (m + nev) / 2;
            const int p = m - b * std::max(1, (m - p_want) / b);
            const int q = p + b;
            std::vector<double> C((size_t)(m + b) * q, 0.0);
            for (int a = 0; a < m; ++a)
                for (int c = 0; c < p; ++c) C[(size_t)a * q + c] = Sv[(size_t)a * m + order[c]];
            for (int x = 0; x < b; ++x) C[(size_t)(m + x) * q + p + x] = 1.0;
            if ((st = S.put(S.dM, C.data(), C.size())) != SPMM_OK) return st;
            float* Vn = S.V[1 - cur_buf];
            if ((st = S.nn(Vc, S.VL, m + b, S.dM, q, 0.0, 1.0, Vn, S.VL)) != SPMM_OK) return st;
            cur_buf = 1 - cur_buf;
            Vc = Vn;
            std::fill(T.begin(), T.end(), 0.0);
            for (int c = 0; c < p; ++c) {
                t(c, c) = theta[order[c]];
                for (int x = 0; x < b; ++x) {
                    double v = 0.0;
                    for (int y = 0; y < b; ++y) v += E[(size_t)x * b + y] * Sv[(size_t)(m - b + y) * m + order[c]];
                    t(p + x, c) = v;
                    t(c, p + x) = v;
                }
            }
            cur = p;
            ++restarts;
        }
        for (int i = 0; i < nev; ++i) {
            const double th = theta[order[i]];
            evals[i] = th;
            if (resid) resid[i] = th != 0.0 ? rnorm[i] / std::fabs(th) : rnorm[i];
        }
        if (evecs) {
            std::vector<double> C((size_t)m * nev);
            for (int a = 0; a < m; ++a)
                for (int c = 0; c < nev; ++c) C[(size_t)a * nev + c] = Sv[(size_t)a * m + order[c]];
            if ((st = S.put(S.dM, C.data(), C.size())) != SPMM_OK) return st;
            if ((st = S.nn(Vc, S.VL, m, S.dM, nev, 0.0, 1.0, evecs, spmm::row_major(ldvec))) != SPMM_OK) return st;
        }
        if ((st = S.sync("eigensolver")) != SPMM_OK) return st;
        double dense_ms = 0.0;
        if ((st = S.dense_ms(dense_ms)) != SPMM_OK) return st;
        if (info) {
            info->n_converged = n_conv;
            info->restarts = restarts;
            info->n_spmm = S.n_spmm;
            info->spmm_ms = S.spmm_ms;
            info->total_ms =
                std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
            info->max_dim = m;
            info->block = b;
            info->dense_ms = dense_ms;
            info->dense_bytes = S.dense_bytes;
            info->n_reorth = S.n_second_pass;
            info->n_orth = S.n_first_pass;
        }
        if (n_conv < nev)
            return fail(SPMM_ENOTCONV, std::to_string(n_conv) + " of " + std::to_string(nev) +
                                           " eigenpairs converged in " + std::to_string(max_restarts) + " restarts");
        return SPMM_OK;
    } catch (const std::exception& ex) {
        return fail(SPMM_ENOMEM, ex.what());
    }
}

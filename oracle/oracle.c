/*
 * ORACLE -- test infrastructure only.
 *
 * Plain, slow, obviously correct CPU reference for what the GPU path
 * computes.  Only the tests, the smoke check and the benchmark's CPU
 * baseline may call this code; the product library never links it, and the
 * two share no source.  Built with -O2 -ffp-contract=off so that every
 * floating-point operation is one IEEE operation in the written order
 * (and -fopenmp for the baseline's multi-threaded leg, which only spreads
 * independent rows over threads).
 *
 * Contents
 *   - SpMM  Y = A X  in FP64, row by row (Algorithm 1: the output starts at
 *     zero and every non-zero (r, c, v) adds v * X[c, :] to Y[r, :]; SpMV is
 *     the one-column case).
 *   - y = A^T x in FP64 (scatter form), for PageRank on directed graphs.
 *   - BF16 and OCP FP8-E4M3 encoders/decoders, written from the format
 *     definitions (nearest representable value, ties to even).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <string.h>

/* Y[i - r0][:] = sum over row i of val * X[col][:], rows r0 <= i < r1, FP64. */
void oracle_spmm_rows_f32x(int64_t r0, int64_t r1, const int64_t* row_ptr, const int32_t* col,
                           const float* val, const float* X, int64_t k, int64_t ldx,
                           double* Y, int64_t ldy) {
    for (int64_t i = r0; i < r1; ++i) {
        for (int64_t j = 0; j < k; ++j) {
            double acc = 0.0;
            for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
                double v = val ? (double)val[p] : 1.0;
                acc += v * (double)X[(int64_t)col[p] * ldx + j];
            }
            Y[(i - r0) * ldy + j] = acc;
        }
    }
}

/* Same, with X already in FP64 (e.g. a dequantised matrix). */
void oracle_spmm_rows_f64x(int64_t r0, int64_t r1, const int64_t* row_ptr, const int32_t* col,
                           const float* val, const double* X, int64_t k, int64_t ldx,
                           double* Y, int64_t ldy) {
    for (int64_t i = r0; i < r1; ++i) {
        for (int64_t j = 0; j < k; ++j) {
            double acc = 0.0;
            for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
                double v = val ? (double)val[p] : 1.0;
                acc += v * X[(int64_t)col[p] * ldx + j];
            }
            Y[(i - r0) * ldy + j] = acc;
        }
    }
}

/* Selected rows only: Y[s][:] = (A X)[rows[s]][:], FP64. */
void oracle_spmm_sel_f32x(int64_t nsel, const int64_t* rows, const int64_t* row_ptr,
                          const int32_t* col, const float* val, const float* X, int64_t k,
                          int64_t ldx, double* Y) {
    for (int64_t s = 0; s < nsel; ++s)
        oracle_spmm_rows_f32x(rows[s], rows[s] + 1, row_ptr, col, val, X, k, ldx, Y + s * k, k);
}

/* The second leg of the CPU baseline: oracle_spmm_sel_f32x with the
   selected rows shared out over the host threads (OpenMP).  Rows are
   independent and each is summed by one thread in the written order, so the
   result equals the single-threaded one bit for bit.  Returns the number of
   threads used. */
int oracle_spmm_sel_f32x_omp(int64_t nsel, const int64_t* rows, const int64_t* row_ptr,
                             const int32_t* col, const float* val, const float* X, int64_t k,
                             int64_t ldx, double* Y) {
    int used = 1;
    #pragma omp parallel
    {
        #pragma omp single
        used = omp_get_num_threads();
        #pragma omp for schedule(dynamic, 16)
        for (int64_t s = 0; s < nsel; ++s)
            oracle_spmm_rows_f32x(rows[s], rows[s] + 1, row_ptr, col, val, X, k, ldx, Y + s * k, k);
    }
    return used;
}

/* y = A^T x in FP64: every stored (r, c, v) adds v * x[r] to y[c]. */
void oracle_spmv_t_f64(int64_t n_rows, int64_t n_cols, const int64_t* row_ptr, const int32_t* col,
                       const float* val, const double* x, double* y) {
    memset(y, 0, sizeof(double) * (size_t)n_cols);
    for (int64_t r = 0; r < n_rows; ++r)
        for (int64_t p = row_ptr[r]; p < row_ptr[r + 1]; ++p)
            y[col[p]] += (val ? (double)val[p] : 1.0) * x[r];
}

/* ----------------------------------------------------------------- BF16 */
/*
 * BF16 keeps the sign, the 8 exponent bits and the top 7 fraction bits of
 * an FP32 value.  Every BF16 value is therefore an FP32 value whose low 16
 * bits are zero.  Encoding a finite x picks, of the two BF16 values that
 * bracket it (truncation toward zero, and the next one away from zero), the
 * nearer; a tie goes to the one whose last kept fraction bit is 0.  Values
 * beyond the largest finite BF16 round to infinity as in IEEE arithmetic.
 * NaN stays NaN (quiet, sign kept).
 */
static uint16_t bf16_from_f32(float x) {
    uint32_t b;
    memcpy(&b, &x, 4);
    if ((b & 0x7F800000u) == 0x7F800000u && (b & 0x007FFFFFu)) return (uint16_t)((b >> 16) | 0x0040u);
    uint32_t toward_zero = b >> 16;      /* truncated magnitude, same sign  */
    uint32_t rest = b & 0xFFFFu;         /* distance past it, in FP32 ulps   */
    if (rest > 0x8000u) return (uint16_t)(toward_zero + 1);
    if (rest < 0x8000u) return (uint16_t)toward_zero;
    return (uint16_t)((toward_zero & 1u) ? toward_zero + 1 : toward_zero);
}

static float bf16_to_f32(uint16_t h) {
    uint32_t b = (uint32_t)h << 16;
    float x;
    memcpy(&x, &b, 4);
    return x;
}

void oracle_bf16_encode(const float* x, int64_t n, uint16_t* out) {
    for (int64_t i = 0; i < n; ++i) out[i] = bf16_from_f32(x[i]);
}

void oracle_bf16_decode(const uint16_t* h, int64_t n, float* out) {
    for (int64_t i = 0; i < n; ++i) out[i] = bf16_to_f32(h[i]);
}

/* --------------------------------------------------------- FP8 E4M3 (OCP) */
/*
 * OCP 8-bit floating point, E4M3 ("E4M3FN"): 1 sign bit, 4 exponent bits
 * with bias 7, 3 fraction bits.  Exponent field 0 encodes subnormals
 * m * 2^-9 (m = 0..7).  Exponent field e = 1..15 encodes (1 + m/8) * 2^(e-7),
 * except S.1111.111 which is NaN; there are no infinities, so the largest
 * finite magnitude is 1.75 * 2^8 = 448.
 *
 * Encoding (saturating): NaN -> S.1111.111; otherwise the nearest E4M3 value
 * to x, ties to an even fraction, with magnitudes beyond 448 clamped to 448.
 */
float oracle_e4m3_value(uint8_t code) {
    int s = code >> 7, e = (code >> 3) & 15, m = code & 7;
    double v;
    if (e == 15 && m == 7) return NAN;
    if (e == 0) v = ldexp((double)m, -9);
    else v = ldexp(1.0 + m / 8.0, e - 7);
    return (float)(s ? -v : v);
}

static uint8_t e4m3_from_f32(float xf) {
    if (isnan(xf)) return signbit(xf) ? 0xFF : 0x7F;
    uint8_t sign = signbit(xf) ? 0x80 : 0x00;
    double a = fabs((double)xf);
    if (a >= 448.0) return sign | 0x7E;                 /* saturate (also inf) */
    /* spacing of E4M3 values around a: 2^(E-3) in binade [2^E, 2^(E+1)),
       and 2^-9 below the smallest normal 2^-6 */
    int E;
    (void)frexp(a, &E);                                 /* a = f * 2^E, f in [0.5,1) */
    E -= 1;                                             /* a in [2^E, 2^(E+1))       */
    if (a == 0.0 || E < -6) E = -6;
    double q = ldexp(1.0, E - 3);
    double r = nearbyint(a / q) * q;                    /* ties to even multiple     */
    if (r > 448.0) r = 448.0;
    if (r == 0.0) return sign;
    int e;
    (void)frexp(r, &e);
    e -= 1;                                             /* r in [2^e, 2^(e+1))       */
    if (e < -6) {                                       /* subnormal                 */
        int m = (int)(r / ldexp(1.0, -9));
        return sign | (uint8_t)m;
    }
    int m = (int)(r / ldexp(1.0, e) * 8.0) - 8;
    return sign | (uint8_t)((e + 7) << 3) | (uint8_t)m;
}

void oracle_e4m3_encode(const float* x, int64_t n, uint8_t* out) {
    for (int64_t i = 0; i < n; ++i) out[i] = e4m3_from_f32(x[i]);
}

void oracle_e4m3_decode(const uint8_t* c, int64_t n, float* out) {
    for (int64_t i = 0; i < n; ++i) out[i] = oracle_e4m3_value(c[i]);
}

/*
 * Per-column FP8 quantisation of an n x k matrix:
 *   absmax_j = max_i |X[i][j]|,  s_j = 448 / absmax_j  (FP32 division; 1 if
 *   the column is all zero),  Q[i][j] = E4M3(X[i][j] * s_j)  with the
 *   product rounded to FP32 first.
 */
void oracle_fp8_colscale(const float* X, int64_t n, int64_t k, int64_t ldx, float* s) {
    for (int64_t j = 0; j < k; ++j) {
        float m = 0.0f;
        for (int64_t i = 0; i < n; ++i) {
            float a = fabsf(X[i * ldx + j]);
            if (a > m) m = a;
        }
        s[j] = (m > 0.0f) ? 448.0f / m : 1.0f;
    }
}

void oracle_fp8_quantize(const float* X, int64_t n, int64_t k, int64_t ldx, const float* s,
                         uint8_t* Q, int64_t ldq) {
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < k; ++j) {
            volatile float prod = X[i * ldx + j] * s[j];
            Q[i * ldq + j] = e4m3_from_f32(prod);
        }
}

void oracle_bf16_quantize(const float* X, int64_t n, int64_t k, int64_t ldx, uint16_t* Q,
                          int64_t ldq) {
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < k; ++j) Q[i * ldq + j] = bf16_from_f32(X[i * ldx + j]);
}

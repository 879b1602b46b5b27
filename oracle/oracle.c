/*
 * FP64 CPU oracle for the BF16 NN GEMM -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may load this
 * library.  It shares no code with the GPU library and is deliberately plain and slow.
 *
 * Problem (paper, Sec. 2.2 "GEMM Tile Hierarchy" and Sec. 7.1): C = A * B with A an M x K
 * matrix and B a K x N matrix, no transposes.  Here A and B hold BF16 bit patterns,
 * row-major with leading dimensions lda (>= K) and ldb (>= N).
 *
 * The exact definition is computed: every BF16 x BF16 product is exact in FP64 (8-bit
 * significands), and the FP64 sum adds at most K * 2^-53 * D_ij of error, far below every
 * tolerance used against it.  D_ij = sum_k |a_ik| |b_kj| is the normaliser of the
 * accuracy criterion max_ij |C_gpu - C_ref| / D_ij.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#include <fenv.h>

/* BF16 bit pattern -> FP64, exact (BF16 is the top half of an FP32). */
double oracle_bf16_to_f64(uint16_t h) {
    uint32_t u = ((uint32_t)h) << 16;
    float f;
    memcpy(&f, &u, sizeof f);
    return (double)f;
}

/* FP64 -> BF16, round to nearest with ties to even, straight from the FP64 value
 * (8 significant bits, exponent range of FP32, gradual underflow below 2^-126). */
uint16_t oracle_f64_to_bf16_rne(double x) {
    if (isnan(x)) return 0x7FC0;
    uint16_t sign = signbit(x) ? 0x8000 : 0;
    double a = fabs(x);
    if (a == 0.0) return sign;
    int e = ilogb(a);                 /* 2^e <= a < 2^(e+1) */
    if (e < -126) e = -126;           /* subnormal BF16: fixed quantum 2^-133 */
    double q = ldexp(1.0, e - 7);     /* spacing of 8-bit significands in this binade */
    int old = fegetround();
    fesetround(FE_TONEAREST);
    double r = nearbyint(a / q) * q;  /* a/q is exact: a power-of-two scaling */
    fesetround(old);
    if (r >= ldexp(1.0, 128)) return sign | 0x7F80;   /* overflow to infinity */
    float f = (float)r;               /* exact: r has at most 8 significant bits */
    uint32_t u;
    memcpy(&u, &f, sizeof u);
    return (uint16_t)(sign | ((u >> 16) & 0x7FFF));
}

/* C_ref[i][j] = sum_k a_ik b_kj and D[i][j] = sum_k |a_ik| |b_kj|, both in FP64.
 * Either output pointer may be NULL.  Loops in the textbook order i, j, k. */
void oracle_gemm_f64(int64_t M, int64_t N, int64_t K,
                     const uint16_t* A, int64_t lda,
                     const uint16_t* B, int64_t ldb,
                     double* C, int64_t ldc, double* D, int64_t ldd) {
    for (int64_t i = 0; i < M; ++i) {
        for (int64_t j = 0; j < N; ++j) {
            double s = 0.0, d = 0.0;
            for (int64_t k = 0; k < K; ++k) {
                double a = oracle_bf16_to_f64(A[i * lda + k]);
                double b = oracle_bf16_to_f64(B[k * ldb + j]);
                s += a * b;
                d += fabs(a) * fabs(b);
            }
            if (C) C[i * ldc + j] = s;
            if (D) D[i * ldd + j] = d;
        }
    }
}

/* The same definition evaluated only at n chosen entries (rows[t], cols[t]). */
void oracle_gemm_entries(int64_t M, int64_t N, int64_t K,
                         const uint16_t* A, int64_t lda,
                         const uint16_t* B, int64_t ldb,
                         int64_t n, const int64_t* rows, const int64_t* cols,
                         double* c_out, double* d_out) {
    (void)M; (void)N;
    for (int64_t t = 0; t < n; ++t) {
        int64_t i = rows[t], j = cols[t];
        double s = 0.0, d = 0.0;
        for (int64_t k = 0; k < K; ++k) {
            double a = oracle_bf16_to_f64(A[i * lda + k]);
            double b = oracle_bf16_to_f64(B[k * ldb + j]);
            s += a * b;
            d += fabs(a) * fabs(b);
        }
        c_out[t] = s;
        d_out[t] = d;
    }
}

/* Accuracy criterion: max over entries of |C_gpu - C_ref| / D.  Where D == 0 the
 * reference is exactly 0 and the GPU value must be exactly 0 as well; any such
 * violation is counted in *zero_violations (and does not enter the maximum). */
double oracle_scaled_err(int64_t n, const double* c_gpu, const double* c_ref,
                         const double* d, int64_t* argmax, int64_t* zero_violations) {
    double worst = 0.0;
    int64_t where = -1, bad = 0;
    for (int64_t t = 0; t < n; ++t) {
        double diff = fabs(c_gpu[t] - c_ref[t]);
        if (d[t] == 0.0) {
            if (c_gpu[t] != 0.0 || isnan(c_gpu[t])) ++bad;
            continue;
        }
        double e = diff / d[t];
        if (isnan(e) || e > worst) {
            worst = isnan(e) ? INFINITY : e;
            where = t;
        }
    }
    if (argmax) *argmax = where;
    if (zero_violations) *zero_violations = bad;
    return worst;
}

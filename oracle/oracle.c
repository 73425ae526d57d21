/*
 * CPU oracle for the streaming Level-1/Level-2 BLAS operations of
 * A. Singh and C. Bassoy, "High Performance Level-1 and Level-2 BLAS"
 * (arXiv 2108.02025).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously
 * correct statement of what the GPU library computes.  Only the test suite,
 * the package smoke check and the CPU-baseline leg of the benchmark may
 * load it.  It shares no code, header, table or constant with the GPU
 * library, and the GPU library never calls it.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no FMA contraction, no
 * fast-math, no reassociation).  Every floating-point sum below is evaluated
 * strictly left to right in IEEE binary64 with round-to-nearest-even.
 *
 * Conventions (from the paper's section 1.1 notation and section 3.1
 * problem definitions):
 *   - A is an m x n matrix with leading dimension lda.  Row-major element
 *     (i, j) lives at A[i*lda + j]; column-major at A[i + j*lda].
 *   - op N:  c (length m) += A x  (x has length n).
 *     op T:  c (length n) += A^T x (x has length m).
 *   - Every operation sums the elementary products first, starting from
 *     +0.0 in ascending index order, and adds the initial output value once,
 *     at the end (section 3.1, the DOT, GEM and GEMV definitions all say the
 *     initial value is added "in the end").
 *   - The elementary products are rounded on their own (the definitions
 *     name separate elementary multiplications and additions), hence no FMA.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_ROW_MAJOR 0
#define ORC_COL_MAJOR 1
#define ORC_OP_N 0
#define ORC_OP_T 1

int32_t orc_version(void) { return 1; }

/* Element (i, j) of an m x n matrix stored in the given layout. */
static double elem(const double* A, int32_t layout, int64_t lda, int64_t i, int64_t j)
{
    return layout == ORC_ROW_MAJOR ? A[i * lda + j] : A[i + j * lda];
}

/*
 * GEMV, section 3.1 (Definition GEMV): c_i += sum_j A_ij x_j, summed over j
 * first, initial c_i added last.  Section 4.1 (Algorithm 1, column-major)
 * and section 4.2 (Algorithm 2, row-major) reach the same sums; the layout
 * only changes where A_ij is stored.
 *
 * op T uses the same definition on A^T: c_j += sum_i A_ij x_i.  The loop
 * below runs i outer and j inner over a private vector t so that a
 * row-major A is read with stride one; for every j the products are still
 * added in ascending i, starting from +0.0, which is the same sum as the
 * j-outer statement of the definition.
 */
int32_t orc_gemv(int32_t layout, int32_t op, int64_t m, int64_t n,
                 const double* A, int64_t lda, const double* x, double* c)
{
    if (m < 0 || n < 0) return -1;
    if (op == ORC_OP_N) {
        for (int64_t i = 0; i < m; ++i) {
            double t = 0.0;
            for (int64_t j = 0; j < n; ++j) {
                double p = elem(A, layout, lda, i, j) * x[j];
                t = t + p;
            }
            c[i] = c[i] + t;
        }
        return 0;
    }
    if (op != ORC_OP_T) return -1;
    double* t = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    if (!t) return -2;
    for (int64_t j = 0; j < n; ++j) t[j] = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            double p = elem(A, layout, lda, i, j) * x[i];
            t[j] = t[j] + p;
        }
    }
    for (int64_t j = 0; j < n; ++j) c[j] = c[j] + t[j];
    free(t);
    return 0;
}

/*
 * Selected outputs of GEMV (same definition as orc_gemv), for checking a
 * sample of a large result one entry at a time.  out[k] receives
 * c0[k] + sum of products for output index idx[k].
 */
int32_t orc_gemv_entries(int32_t layout, int32_t op, int64_t m, int64_t n,
                         const double* A, int64_t lda, const double* x,
                         const int64_t* idx, int64_t count, const double* c0,
                         double* out)
{
    for (int64_t k = 0; k < count; ++k) {
        int64_t r = idx[k];
        double t = 0.0;
        if (op == ORC_OP_N) {
            if (r < 0 || r >= m) return -1;
            for (int64_t j = 0; j < n; ++j) {
                double p = elem(A, layout, lda, r, j) * x[j];
                t = t + p;
            }
        } else {
            if (r < 0 || r >= n) return -1;
            for (int64_t i = 0; i < m; ++i) {
                double p = elem(A, layout, lda, i, r) * x[i];
                t = t + p;
            }
        }
        out[k] = c0[k] + t;
    }
    return 0;
}

/*
 * DOT, section 3.1 (Definition DOT): alpha += sum_p x_p y_p, products summed
 * in ascending p from +0.0, the initial alpha added at the end.  Section 4.3
 * (Algorithms 3 and 4) splits the same sum into blocks; the definition is the
 * reference.
 */
double orc_dot(int64_t n, const double* x, const double* y, double alpha)
{
    double t = 0.0;
    for (int64_t p = 0; p < n; ++p) {
        double q = x[p] * y[p];
        t = t + q;
    }
    return alpha + t;
}

/*
 * GER, section 3.1 (Definition GEM, the outer product): C_ij += x_i y_j.
 * Each output has exactly one elementary product, rounded, then the initial
 * C_ij is added (two roundings).  Section 4.2 (Algorithm 2) updates the same
 * entries in row order.
 */
int32_t orc_ger(int32_t layout, int64_t m, int64_t n, const double* x,
                const double* y, double* C, int64_t ldc)
{
    if (m < 0 || n < 0) return -1;
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            double p = x[i] * y[j];
            double* cij = layout == ORC_ROW_MAJOR ? &C[i * ldc + j] : &C[i + j * ldc];
            *cij = *cij + p;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Storage formats for the precision form.  The paper leaves the element
 * width generic (section 2, S_data); the narrow formats below follow their
 * published definitions:
 *   bfloat16: the upper 16 bits of an IEEE binary32 (1 sign, 8 exponent,
 *             7 fraction bits), round-to-nearest-even.
 *   E4M3FN (OCP 8-bit floating point, E4M3 variant): 1 sign, 4 exponent
 *             bits with bias 7, 3 fraction bits; exponent field 0 encodes
 *             subnormals of value M * 2^-9; S.1111.111 is NaN; there is no
 *             infinity; the largest finite magnitude is 448.
 * The encoders here work on exact binary64 values and ldexp, so no step
 * depends on bit tricks that a GPU implementation might share.
 * ------------------------------------------------------------------------ */

static uint32_t f32_bits(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }
static float f32_from_bits(uint32_t u) { float f; memcpy(&f, &u, 4); return f; }

/* Round a non-negative exact value v (v = k/2 granularity allowed) to the
 * nearest integer, ties to even.  v is exact in binary64 here. */
static double rne_integer(double v)
{
    double fl = floor(v);
    double fr = v - fl; /* exact: fl and v share the binade or fl = 0 */
    if (fr > 0.5) return fl + 1.0;
    if (fr < 0.5) return fl;
    return fmod(fl, 2.0) == 0.0 ? fl : fl + 1.0;
}

float orc_bf16_to_f32(uint16_t b) { return f32_from_bits(((uint32_t)b) << 16); }

uint16_t orc_bf16_from_f32(float f)
{
    uint32_t u = f32_bits(f);
    uint16_t sign = (uint16_t)((u >> 16) & 0x8000u);
    if (isnan(f)) return (uint16_t)(sign | 0x7FC0u);
    double v = fabs((double)f);
    if (v == 0.0 || isinf(f)) return (uint16_t)(u >> 16);
    /* Quantum of bfloat16 at v: 8 significant bits, minimum exponent -126,
     * subnormal quantum 2^-133. */
    int e;
    frexp(v, &e);            /* v = f * 2^e, f in [0.5, 1): floor(log2 v) = e-1 */
    int q = (e - 1) - 7;
    if (q < -133) q = -133;
    double k = rne_integer(ldexp(v, -q));
    double r = ldexp(k, q);
    /* r is a bfloat16 value (or 2^128 on overflow); binary32 holds it. */
    float rf = r >= 0x1p128 ? INFINITY : (float)r;
    return (uint16_t)(sign | (f32_bits(rf) >> 16));
}

float orc_e4m3_to_f32(uint8_t code)
{
    int s = code >> 7;
    int E = (code >> 3) & 0xF;
    int M = code & 0x7;
    double v;
    if (E == 15 && M == 7) return NAN;
    if (E == 0) v = ldexp((double)M, -9);
    else v = ldexp((double)(8 + M), E - 10);
    return (float)(s ? -v : v);
}

/* Round to E4M3FN, nearest-even, saturating magnitudes above 448 to 448. */
static uint8_t e4m3_from_f64(double d, int negative)
{
    uint8_t sign = negative ? 0x80 : 0x00;
    if (isnan(d)) return (uint8_t)(sign | 0x7F);
    double v = fabs(d);
    if (v >= 448.0) return (uint8_t)(sign | 0x7E);
    if (v < 0x1p-6) {
        /* Subnormal range, quantum 2^-9; k = 8 lands exactly on 2^-6, whose
         * code is 0x08, so the code is k itself. */
        double k = rne_integer(ldexp(v, 9));
        return (uint8_t)(sign | (uint8_t)k);
    }
    int e;
    frexp(v, &e);
    int ex = e - 1;                          /* v in [2^ex, 2^(ex+1)) */
    double k = rne_integer(ldexp(v, 3 - ex)); /* in [8, 16] */
    if (k == 16.0) { k = 8.0; ex += 1; }
    int field = ex + 7;
    if (field > 15 || (field == 15 && k - 8.0 > 6.0)) return (uint8_t)(sign | 0x7E);
    return (uint8_t)(sign | (uint8_t)(field << 3) | (uint8_t)(k - 8.0));
}

uint8_t orc_e4m3_from_f32(float f) { return e4m3_from_f64((double)f, (int)(f32_bits(f) >> 31)); }

/*
 * Per-row scaled quantisation (precision form; the paper is silent on it).
 *   amax_i = max_j |a_ij| over the non-NaN entries of row i.
 *   bfloat16: s_i = 2^floor(log2 amax_i), so a/s is exact and q carries the
 *             same rounding error as a plain bfloat16 cast.
 *   E4M3:     s_i = fl32(amax_i / 448).
 *   A row whose amax is 0, infinite or NaN gets s_i = 1.
 *   q_ij = encode(fl32(a_ij / s_i)).
 * q = 2 selects bfloat16 (2-byte codes), q = 3 selects E4M3 (1-byte codes),
 * matching the dtype numbering of the library.
 */
int32_t orc_quantize_rows(int32_t q, int64_t m, int64_t n, const float* A,
                          int64_t lda, void* Aq, int64_t ldq, float* scales)
{
    if (q != 2 && q != 3) return -1;
    for (int64_t i = 0; i < m; ++i) {
        float amax = 0.0f;
        for (int64_t j = 0; j < n; ++j) {
            float a = fabsf(A[i * lda + j]);
            if (!isnan(a) && a > amax) amax = a;
        }
        float s;
        if (amax == 0.0f || isinf(amax)) {
            s = 1.0f;
        } else if (q == 2) {
            int e;
            frexp((double)amax, &e);
            s = (float)ldexp(1.0, e - 1);
        } else {
            s = amax / 448.0f;
            if (s == 0.0f) s = 1.0f; /* amax below 448 * 2^-150 */
        }
        scales[i] = s;
        for (int64_t j = 0; j < n; ++j) {
            float v = A[i * lda + j] / s;
            if (q == 2) ((uint16_t*)Aq)[i * ldq + j] = orc_bf16_from_f32(v);
            else ((uint8_t*)Aq)[i * ldq + j] = orc_e4m3_from_f32(v);
        }
    }
    return 0;
}

/*
 * Dequantised GEMV reference: c_i += s_i * sum_j q_ij x_j, evaluated in
 * binary64.  Every decoded q has at most 8 significant bits and x is
 * binary32, so each product is exact and only the sum rounds.
 */
int32_t orc_gemv_q(int32_t q, int64_t m, int64_t n, const void* Aq, int64_t ldq,
                   const float* scales, const float* x, double* c)
{
    if (q != 2 && q != 3) return -1;
    for (int64_t i = 0; i < m; ++i) {
        double t = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            double a = q == 2 ? (double)orc_bf16_to_f32(((const uint16_t*)Aq)[i * ldq + j])
                              : (double)orc_e4m3_to_f32(((const uint8_t*)Aq)[i * ldq + j]);
            double p = a * (double)x[j];
            t = t + p;
        }
        double st = (double)scales[i] * t;
        c[i] = c[i] + st;
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Exact dot product of binary32 vectors (reference for the compensated
 * DOT).  Each product x_i*y_i of two binary32 numbers has at most 48
 * significant bits and is therefore exact in binary64.  The products are
 * accumulated exactly in a long fixed-point accumulator (32-bit digits held
 * in signed 64-bit cells, bit 0 of the accumulator weighing 2^-1074), and
 * the total is rounded once, to nearest-even, into binary64.
 * ------------------------------------------------------------------------ */

#define LACC_DIGITS 72 /* 72 * 32 = 2304 bits >= 1074 + 1024 + carries */

typedef struct { int64_t d[LACC_DIGITS]; int64_t pending; } lacc;

static void lacc_norm(lacc* a)
{
    for (int k = 0; k < LACC_DIGITS - 1; ++k) {
        int64_t carry = a->d[k] >> 32; /* arithmetic shift: floor division */
        a->d[k] -= carry * ((int64_t)1 << 32);
        a->d[k + 1] += carry;
    }
    a->pending = 0;
}

static void lacc_add(lacc* a, double v)
{
    if (v == 0.0) return;
    int e;
    double f = frexp(fabs(v), &e);                /* |v| = f * 2^e */
    uint64_t M = (uint64_t)ldexp(f, 53);          /* exact 53-bit integer */
    int64_t pos = (int64_t)e - 53 + 1074;         /* weight of M's bit 0 */
    if (pos < 0) { M >>= -pos; pos = 0; }         /* only for subnormal v: exact */
    int k = (int)(pos / 32), r = (int)(pos % 32);
    unsigned __int128 w = ((unsigned __int128)M) << r;
    int64_t sgn = v < 0 ? -1 : 1;
    for (int t = 0; t < 3 && w; ++t, w >>= 32)
        a->d[k + t] += sgn * (int64_t)(uint64_t)(w & 0xFFFFFFFFu);
    if (++a->pending >= ((int64_t)1 << 29)) lacc_norm(a);
}

/* Round the accumulator to binary64 (nearest-even).  The result is assumed
 * to be zero or a normal binary64 number, which holds for sums of binary32
 * products. */
static double lacc_round(lacc* a)
{
    lacc_norm(a);
    int neg = a->d[LACC_DIGITS - 1] < 0;
    uint32_t mag[LACC_DIGITS];
    if (neg) { /* two's complement negate over the 32-bit digits */
        uint64_t carry = 1;
        for (int k = 0; k < LACC_DIGITS; ++k) {
            uint64_t t = (uint64_t)(~(uint32_t)a->d[k]) + carry;
            mag[k] = (uint32_t)t;
            carry = t >> 32;
        }
    } else {
        for (int k = 0; k < LACC_DIGITS; ++k) mag[k] = (uint32_t)a->d[k];
    }
    int top = LACC_DIGITS - 1;
    while (top >= 0 && mag[top] == 0) --top;
    if (top < 0) return 0.0;
    /* Gather the leading 96 bits into a 128-bit window plus a sticky bit. */
    unsigned __int128 win = 0;
    int lowest = top - 2; /* digits top, top-1, top-2 */
    for (int k = top; k >= lowest; --k) win = (win << 32) | (k >= 0 ? mag[k] : 0);
    int sticky = 0;
    for (int k = lowest - 1; k >= 0; --k) if (mag[k]) { sticky = 1; break; }
    int nbits = 0;
    for (unsigned __int128 t = win; t; t >>= 1) ++nbits;
    int drop = nbits - 53; /* >= 96-32-53 > 0 since the top digit is non-zero */
    unsigned __int128 keep = win >> drop;
    unsigned __int128 rem = win - (keep << drop);
    unsigned __int128 half = ((unsigned __int128)1) << (drop - 1);
    if (rem > half || (rem == half && (sticky || (keep & 1)))) keep += 1;
    int64_t exp2 = (int64_t)lowest * 32 + drop - 1074;
    double r = ldexp((double)(uint64_t)keep, (int)exp2); /* keep <= 2^53: exact */
    return neg ? -r : r;
}

/*
 * Exact alpha0 + sum_i x_i y_i, rounded once to binary64.  If absval is
 * non-zero the sum of |x_i y_i| (and |alpha0|) is returned instead, which
 * gives the exact condition number 2 sum|x_i y_i| / |sum x_i y_i| of the
 * dot product.
 */
double orc_dot_exact_f32(int64_t n, const float* x, const float* y, float alpha0, int32_t absval)
{
    lacc* a = (lacc*)calloc(1, sizeof(lacc));
    if (!a) return NAN;
    for (int64_t i = 0; i < n; ++i) {
        double p = (double)x[i] * (double)y[i]; /* exact */
        lacc_add(a, absval ? fabs(p) : p);
    }
    lacc_add(a, absval ? fabs((double)alpha0) : (double)alpha0);
    double r = lacc_round(a);
    free(a);
    return r;
}

/* Exact sum of binary64 values, rounded once (used to pin the accumulator
 * and for exact references of short binary64 sums whose terms are exact). */
double orc_sum_exact_f64(int64_t n, const double* v)
{
    lacc* a = (lacc*)calloc(1, sizeof(lacc));
    if (!a) return NAN;
    for (int64_t i = 0; i < n; ++i) lacc_add(a, v[i]);
    double r = lacc_round(a);
    free(a);
    return r;
}

/*
 * Microscaling (OCP Microscaling Formats specification v1.0): each row is
 * cut into blocks of 32 consecutive elements (the last block of a row may
 * be shorter); a block stores one shared scale X in E8M0 (X = 2^(code-127),
 * code 255 is NaN) and its elements P_j in E4M3 (MXFP8) or E2M1 (MXFP4);
 * element j decodes to X * P_j.
 *
 * E2M1: sign, 2 exponent bits (bias 1), 1 mantissa bit, no infinities or
 * NaN; the eight magnitudes are 0, 0.5, 1, 1.5, 2, 3, 4, 6.
 */
double orc_e8m0_to_f64(uint8_t code) { return code == 255 ? NAN : ldexp(1.0, (int)code - 127); }

double orc_e2m1_to_f64(uint8_t code)
{
    const int s = (code >> 3) & 1, e = (code >> 1) & 3, mbit = code & 1;
    const double mag = e == 0 ? 0.5 * mbit : ldexp(1.0 + 0.5 * mbit, e - 1);
    return s ? -mag : mag;
}

/* Round to the nearest of the eight magnitudes; a tie goes to the code with
 * an even last bit; beyond 6 the magnitude saturates to 6.  The sign is
 * kept (so -0.0 and small negatives give the code 8, negative zero). */
uint8_t orc_e2m1_from_f64(double v)
{
    const int neg = signbit(v) ? 1 : 0;
    const double a = fabs(v);
    int best = 0;
    double bestd = INFINITY;
    for (int c = 0; c < 8; ++c) {
        const double d = fabs(a - orc_e2m1_to_f64((uint8_t)c));
        if (d < bestd || (d == bestd && (c & 1) == 0)) {
            best = c;
            bestd = d;
        }
    }
    if (a > 6.0) best = 7;
    return (uint8_t)((neg << 3) | best);
}

/*
 * MX quantisation of a row-major m x n binary32 matrix, blocks of 32 along
 * each row (scale rule of the specification's conversion section):
 *   a block with a non-finite element: X code 255 (NaN), element codes 0;
 *   a block of zeros: X code 0, element codes of signed zero;
 *   otherwise E = floor(log2 amax) and code = clamp(E - emax + 127, 0, 254)
 *   with emax = 8 (E4M3, largest normal 448 = 1.75 * 2^8) or 2 (E2M1,
 *   largest 6 = 1.5 * 2^2); P_j = encode(a_j / X), a_j / X exact in binary64,
 *   rounded to nearest even and saturated.
 * q = 4 selects MXFP8 (E4M3 codes, one byte each, row stride ldq bytes);
 * q = 5 selects MXFP4 (E2M1 codes, element 2k in the low nibble and 2k+1 in
 * the high nibble of byte k of the row; an unused high nibble is 0).
 * Scales: S[i * lds + b] for block b of row i.
 */
int32_t orc_quantize_mx(int32_t q, int64_t m, int64_t n, const float* A, int64_t lda,
                        uint8_t* Q, int64_t ldq, uint8_t* S, int64_t lds)
{
    if (q != 4 && q != 5) return -1;
    const int emax = q == 4 ? 8 : 2;
    const int64_t nb = (n + 31) / 32;
    for (int64_t i = 0; i < m; ++i) {
        if (q == 5)
            for (int64_t k = 0; k < (n + 1) / 2; ++k) Q[i * ldq + k] = 0;
        for (int64_t b = 0; b < nb; ++b) {
            const int64_t j0 = 32 * b, j1 = j0 + 32 < n ? j0 + 32 : n;
            int finite = 1;
            double amax = 0.0;
            for (int64_t j = j0; j < j1; ++j) {
                const double a = (double)A[i * lda + j];
                if (!isfinite(a)) finite = 0;
                else if (fabs(a) > amax) amax = fabs(a);
            }
            int code;
            if (!finite) {
                code = 255;
            } else if (amax == 0.0) {
                code = 0;
            } else {
                int ex;
                frexp(amax, &ex);              /* amax in [2^(ex-1), 2^ex) */
                code = (ex - 1) - emax + 127;
                if (code < 0) code = 0;
                if (code > 254) code = 254;
            }
            S[i * lds + b] = (uint8_t)code;
            for (int64_t j = j0; j < j1; ++j) {
                const double a = (double)A[i * lda + j];
                uint8_t c = 0;
                if (code != 255) {
                    const double v = ldexp(a, 127 - code);
                    c = q == 4 ? e4m3_from_f64(v, signbit(v) ? 1 : 0) : orc_e2m1_from_f64(v);
                }
                if (q == 4) Q[i * ldq + j] = c;
                else Q[i * ldq + j / 2] |= (uint8_t)(c << (4 * (j & 1)));
            }
        }
    }
    return 0;
}

static double mx_element(int32_t q, const uint8_t* Qrow, int64_t j)
{
    if (q == 4) return (double)orc_e4m3_to_f32(Qrow[j]);
    return orc_e2m1_to_f64((uint8_t)((Qrow[j / 2] >> (4 * (j & 1))) & 15));
}

/*
 * Dequantised MX GEMV reference: c_i += sum_j X_i,j/32 * P_ij * x_j in
 * binary64, ascending j from +0.0, the initial c_i added last.  Each
 * product has at most 4 + 24 significant bits times a power of two, so it
 * is exact and only the sum rounds.
 */
int32_t orc_gemv_mx(int32_t q, int64_t m, int64_t n, const uint8_t* Q, int64_t ldq, const uint8_t* S,
                    int64_t lds, const float* x, double* c)
{
    if (q != 4 && q != 5) return -1;
    for (int64_t i = 0; i < m; ++i) {
        double t = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            const double X = orc_e8m0_to_f64(S[i * lds + j / 32]);
            const double p = X * mx_element(q, Q + i * ldq, j);
            t += p * (double)x[j];
        }
        c[i] = c[i] + t;
    }
    return 0;
}

/*
 * CPU oracle for systematic MDS erasure coding over GF(2^w).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * definition of what the accelerated path must compute.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  It shares
 * no code, header, table or helper with the library under
 * paper_1709_00178_amd/: the ring lift, the XOR schedule and every kernel live
 * there and nowhere here.
 *
 * What is computed (Detchart & Lacan, "Improving the coding speed of erasure
 * codes with polynomial ring transforms"):
 *   - Sec. II-A: the field F_{2^w} = F_2[x]/(p(x)), p irreducible of degree w.
 *     An element is an integer whose bit t is the coefficient of x^t.
 *     Multiplication here is the classic log/antilog table method, with the
 *     smallest primitive element as the table base.
 *   - Sec. II-B / Sec. III: a systematic MDS code whose parity part is a
 *     Cauchy matrix; any square submatrix of the parity part is invertible.
 *     The paper's "generalized Cauchy" points and scalings are never printed;
 *     the plain Cauchy matrix C[i][j] = 1 / (X_i + Y_j) with X_i = i (i < m)
 *     and Y_j = m + j (j < k) is used.  Any other parity matrix may be given.
 *   - Sec. III: each block of the code is handled as w chunks ("slices") of S
 *     bytes.  Symbol (o, b) of a block, for byte offset o and bit b, has
 *     coefficient t equal to bit b of byte o of slice t.
 *   - Encoding: parity_i = sum_j C[i][j] * data_j, symbol by symbol.
 *   - Decoding (Sec. IV-C: the decoding matrix depends on the loss pattern):
 *     take the first k surviving blocks, invert the matching k x k rows of the
 *     systematic generator [I; C] by Gauss-Jordan elimination, recover the
 *     data symbol by symbol and re-encode any erased parity.
 *
 * Threads: byte offsets are split across OpenMP threads, as the paper splits
 * the symbols across pthreads (Sec. IV-B); each thread owns disjoint bytes.
 *
 * Parity is pinned (tests/test_oracle.py) against an independent shift-and-
 * reduce multiply, brute-force field axioms, the binary-matrix form of the
 * same map, closed forms (XOR parity, multiply by x^s), and recovery from
 * every erasure pattern.  The parity bytes of the paper's own generator are
 * "parity unpinned": the paper prints no codeword and no matrix.
 *
 * OR_MUTANT (default 0) plants one known mistake per nonzero value, so that
 * tests/test_oracle_mutants.py can show each of them is caught by the pins.
 * A normal build compiles every mutant branch away.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef OR_MUTANT
#define OR_MUTANT 0
#endif

#define OR_OK 0
#define OR_EINVAL -1
#define OR_ENOTIRRED -2
#define OR_ETOOLONG -3
#define OR_ESINGULAR -4
#define OR_ETOOMANY -5
#define OR_ENOMEM -6

#define OR_WMAX 16

typedef struct {
    int w;
    uint32_t p;   /* modulus including the x^w term */
    uint32_t q1;  /* 2^w - 1: order of the multiplicative group */
    uint32_t g;   /* table base: smallest element of order 2^w - 1 */
    uint32_t *exp_t;  /* exp_t[i] = g^i for 0 <= i < 2*q1 */
    uint32_t *log_t;  /* log_t[g^i] = i; log_t[0] unused */
} or_field;

void or_mul_many(const or_field *f, const uint32_t *a, const uint32_t *b, uint32_t *out, size_t n);

/* Multiply a by x and reduce modulo p: one step of the schoolbook method. */
static uint32_t mulx_mod(uint32_t a, int w, uint32_t p) {
    a <<= 1;
    if (a >> w & 1u) a ^= p;
    return a;
}

/* Schoolbook product mod p, used only while building the tables. */
static uint32_t slow_mul(uint32_t a, uint32_t b, int w, uint32_t p) {
    uint32_t r = 0;
    for (int i = 0; i < w; ++i) {
        if (b >> i & 1u) r ^= a;
        a = mulx_mod(a, w, p);
    }
    return r;
}

void or_field_free(or_field *f) {
    if (!f) return;
    free(f->exp_t);
    free(f->log_t);
    free(f);
}

/*
 * Build the log/antilog tables for F_2[x]/(p).  Fails with OR_ENOTIRRED when
 * no element has order 2^w - 1, which happens exactly when p is reducible
 * (the multiplicative group of a field is cyclic).
 */
int or_field_create(int w, uint32_t p, or_field **out) {
    if (!out || w < 1 || w > OR_WMAX || (p >> w) != 1u) return OR_EINVAL;
    or_field *f = (or_field *)calloc(1, sizeof(or_field));
    if (!f) return OR_ENOMEM;
    f->w = w;
    f->p = p;
    f->q1 = (1u << w) - 1u;
    f->exp_t = (uint32_t *)malloc(sizeof(uint32_t) * 2u * (f->q1 + 1u));
    f->log_t = (uint32_t *)calloc(f->q1 + 1u, sizeof(uint32_t));
    if (!f->exp_t || !f->log_t) { or_field_free(f); return OR_ENOMEM; }
    if (w == 1) {  /* GF(2): the group is trivial, 1 generates it */
        f->g = 1;
        f->exp_t[0] = f->exp_t[1] = 1;
        f->log_t[1] = 0;
        *out = f;
        return OR_OK;
    }
    for (uint32_t g = 2; g <= f->q1; ++g) {
        /* order of g: the first i >= 1 with g^i == 1 */
        uint32_t v = g, ord = 1;
        while (v != 1u && ord <= f->q1) {
            v = slow_mul(v, g, w, p);
            ++ord;
            if (v == 0) { ord = f->q1 + 1; break; }  /* zero divisor */
        }
        if (ord == f->q1 || (OR_MUTANT == 1 && g == 2)) { f->g = g; break; }
    }
    if (f->g == 0) { or_field_free(f); return OR_ENOTIRRED; }
    uint32_t v = 1;
    for (uint32_t i = 0; i < 2u * f->q1; ++i) {
        f->exp_t[i] = v;
        if (i < f->q1) f->log_t[v] = i;
        v = slow_mul(v, f->g, w, p);
    }
    *out = f;
    return OR_OK;
}

uint32_t or_field_generator(const or_field *f) { return f->g; }

uint32_t or_mul(const or_field *f, uint32_t a, uint32_t b) {
    if (a == 0 || b == 0) return 0;
    return f->exp_t[f->log_t[a] + f->log_t[b] + (OR_MUTANT == 2)];
}

void or_mul_many(const or_field *f, const uint32_t *a, const uint32_t *b, uint32_t *out, size_t n) {
    for (size_t i = 0; i < n; ++i) out[i] = or_mul(f, a[i], b[i]);
}

uint32_t or_inv(const or_field *f, uint32_t a) {
    if (a == 0) return 0;  /* callers never invert zero */
    return f->exp_t[(f->q1 - f->log_t[a] + (OR_MUTANT == 3)) % f->q1];
}

/* Parity part of the systematic generator: C[i][j] = 1 / (i + (m + j)). */
int or_cauchy(const or_field *f, int k, int m, uint16_t *C) {
    if (k < 1 || m < 0) return OR_EINVAL;
    if ((uint32_t)(k + m) > f->q1 + 1u) return OR_ETOOLONG;
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < k; ++j)
            C[i * k + j] = (uint16_t)or_inv(f, (uint32_t)i ^ (uint32_t)(OR_MUTANT == 4 ? j + 1 : m + j));
    return OR_OK;
}

/* Symbol (o, b) of a bit-sliced block: bit t is bit b of byte o of slice t. */
static uint32_t get_symbol(const uint8_t *blk, int w, size_t S, size_t o, int b) {
    uint32_t u = 0;
    for (int t = 0; t < w; ++t)
        u |= (uint32_t)((blk[(size_t)(OR_MUTANT == 5 ? w - 1 - t : t) * S + o] >> b) & 1u) << t;
    return u;
}

static void put_symbol(uint8_t *blk, int w, size_t S, size_t o, int b, uint32_t u) {
    for (int t = 0; t < w; ++t) {
        uint8_t *byte = &blk[(size_t)t * S + o];
        *byte = (uint8_t)((*byte & ~(1u << b)) | (((u >> t) & 1u) << b));
    }
}

/*
 * out_i = sum_j M[i][j] * in_j for i < rows, j < cols, over symbols in the
 * byte-offset range [o0, o1).  in/out are arrays of block base pointers; each
 * block is w slices of S bytes.
 */
static void matvec_blocks(const or_field *f, int rows, int cols, const uint16_t *M,
                          const uint8_t *const *in, uint8_t *const *out, size_t S,
                          size_t o0, size_t o1, int nthreads) {
    const int w = f->w;
    long long lo = (long long)o0, hi = (long long)o1;
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (long long oo = lo; oo < hi; ++oo) {
        size_t o = (size_t)oo;
        uint32_t u[64];
        for (int b = 0; b < 8; ++b) {
            for (int j = 0; j < cols; ++j) u[j] = get_symbol(in[j], w, S, o, b);
            for (int i = 0; i < rows; ++i) {
                uint32_t acc = 0;
                for (int j = 0; j < cols - (OR_MUTANT == 6 && cols > 1); ++j)
                    acc ^= or_mul(f, M[i * cols + j], u[j]);
                put_symbol(out[i], w, S, o, b, acc);
            }
        }
    }
}

/* Encode m parity blocks from k data blocks with parity matrix C (m x k). */
int or_encode(const or_field *f, int k, int m, const uint16_t *C,
              const uint8_t *const *data, uint8_t *const *parity, size_t S,
              size_t o0, size_t o1, int nthreads) {
    if (!f || !C || !data || !parity || k < 1 || k > 64 || m < 0 || o0 > o1 || o1 > S)
        return OR_EINVAL;
    for (int i = 0; i < m * k; ++i)
        if (C[i] > f->q1) return OR_EINVAL;
    if (nthreads < 1) nthreads = 1;
    matvec_blocks(f, m, k, C, data, parity, S, o0, o1, nthreads);
    return OR_OK;
}

/*
 * Invert the k x k matrix A in place by Gauss-Jordan elimination (pivot: the
 * first nonzero entry at or below the diagonal).  Returns OR_ESINGULAR when
 * some column has no pivot.
 */
int or_invert(const or_field *f, int k, uint16_t *A) {
    uint16_t *I = (uint16_t *)calloc((size_t)k * k, sizeof(uint16_t));
    if (!I) return OR_ENOMEM;
    for (int i = 0; i < k; ++i) I[i * k + i] = 1;
    for (int c = 0; c < k; ++c) {
        int piv = -1;
        for (int r = c; r < k; ++r)
            if (A[r * k + c]) { piv = r; break; }
        if (piv < 0) { free(I); return OR_ESINGULAR; }
        if (piv != c && OR_MUTANT != 7) {
            for (int x = 0; x < k; ++x) {
                uint16_t t = A[c * k + x]; A[c * k + x] = A[piv * k + x]; A[piv * k + x] = t;
                t = I[c * k + x]; I[c * k + x] = I[piv * k + x]; I[piv * k + x] = t;
            }
        }
        uint32_t s = or_inv(f, A[c * k + c]);
        for (int x = 0; x < k; ++x) {
            A[c * k + x] = (uint16_t)or_mul(f, s, A[c * k + x]);
            I[c * k + x] = (uint16_t)or_mul(f, s, I[c * k + x]);
        }
        for (int r = 0; r < k; ++r) {
            if (r == c || A[r * k + c] == 0) continue;
            uint32_t e = A[r * k + c];
            for (int x = 0; x < k; ++x) {
                A[r * k + x] ^= (uint16_t)or_mul(f, e, A[c * k + x]);
                I[r * k + x] ^= (uint16_t)or_mul(f, e, I[c * k + x]);
            }
        }
    }
    memcpy(A, I, sizeof(uint16_t) * (size_t)k * k);
    free(I);
    return OR_OK;
}

/*
 * Recover the erased blocks.  blocks[0..k-1] are data, blocks[k..k+m-1] are
 * parity; the blocks listed in erased[] are outputs, all others are inputs.
 * Survivors are the first k indices not erased.  Data is recovered through the
 * inverse of the survivors' rows of [I; C]; erased parity is then re-encoded
 * from the (complete) data.
 */
int or_decode(const or_field *f, int k, int m, const uint16_t *C,
              const int *erased, int n_erased, uint8_t *const *blocks, size_t S,
              size_t o0, size_t o1, int nthreads) {
    if (!f || !C || !blocks || k < 1 || k > 64 || m < 0 || m > 64 || n_erased < 0 || o0 > o1 ||
        o1 > S)
        return OR_EINVAL;
    if (n_erased > m) return OR_ETOOMANY;
    if (n_erased == 0) return OR_OK;
    if (!erased) return OR_EINVAL;
    int is_erased[128] = {0};
    for (int e = 0; e < n_erased; ++e) {
        if (erased[e] < 0 || erased[e] >= k + m || is_erased[erased[e]]) return OR_EINVAL;
        is_erased[erased[e]] = 1;
    }
    if (nthreads < 1) nthreads = 1;
    int surv[64], ns = 0;
    for (int i = 0; i < k + m && ns < k; ++i)
        if (!is_erased[i]) surv[ns++] = i;
    uint16_t *A = (uint16_t *)calloc((size_t)k * k, sizeof(uint16_t));
    if (!A) return OR_ENOMEM;
    for (int r = 0; r < k; ++r) {
        int g = surv[r];
        for (int c = 0; c < k; ++c)
            A[r * k + c] = (g < k) ? (uint16_t)(g == c)
                                   : C[(g - k) * k + (OR_MUTANT == 9 ? k - 1 - c : c)];
    }
    int rc = or_invert(f, k, A);
    if (rc != OR_OK) { free(A); return rc; }
    /* recover every erased data block: data_j = sum_r Ainv[j][r] * survivor_r */
    const uint8_t *in[64];
    for (int r = 0; r < k; ++r) in[r] = blocks[surv[r]];
    for (int j = 0; j < k; ++j) {
        if (!is_erased[j]) continue;
        uint8_t *outp[1] = {blocks[j]};
        matvec_blocks(f, 1, k, A + (size_t)j * k, in, outp, S, o0, o1, nthreads);
    }
    /* re-encode every erased parity block from the now complete data */
    const uint8_t *dat[64];
    for (int j = 0; j < k; ++j) dat[j] = blocks[j];
    for (int i = 0; i < m; ++i) {
        if (!is_erased[k + i] || OR_MUTANT == 8) continue;
        uint8_t *outp[1] = {blocks[k + i]};
        matvec_blocks(f, 1, k, C + (size_t)i * k, dat, outp, S, o0, o1, nthreads);
    }
    free(A);
    return OR_OK;
}

int or_max_threads(void) {
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * lsh_oracle.c -- plain FP64 CPU oracle for the LSH indexing path.
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the tests, the smoke check and
 * the CPU-baseline leg of the benchmark load this library.  It shares no code,
 * header, table or constant with the GPU library: everything here is written
 * out again from the paper's definitions (Verma & Pratap, "Faster and Space
 * Efficient Indexing for Locality Sensitive Hashing").
 *
 * What it computes, step by step, in the paper's order:
 *   1. decode the stored point values to FP64 (FP32, BF16 or FP8-E4M3FN times
 *      a per-row FP32 scale; every decode is exact in FP64);
 *   2. project: count sketch (Definition "Count Sketch"), higher-order count
 *      sketch (Definition "Higher Order Count Sketch", Eq. eqhcs, padded with
 *      zeros as in Section 6), or the dense Gaussian projection <r, p>
 *      (Definitions of E2LSH and SRP);
 *   3. discretise: floor((alpha*y + b)/w) with alpha = sqrt(m) for CS-E2LSH /
 *      HCS-E2LSH (Definitions CS-E2LSH and HCS-E2LSH) and alpha = 1 for dense
 *      E2LSH (Eq. datar_lsh); sgn(y) = 1 iff y > 0 for the SRP family
 *      (Definitions SRP, CS-SRP, HCS-SRP);
 *   4. concatenate the K codes of each of L tables into one bucket key
 *      (Section 3.1, the (m, tau) index of Indyk and Motwani);
 *   5. store every point in the bucket of its key, per table (Section 3.1);
 *   6. answer a query by the union of its buckets (Section 3.1), re-ranked by
 *      exact distance (Section 6, top-k retrieval).
 *
 * Summation is left to right in ascending coordinate index.  Compile without
 * floating-point contraction (-ffp-contract=off) so every product and sum is
 * rounded separately, exactly as written.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORC_F32 = 0, ORC_BF16 = 1, ORC_FP8 = 2 };
enum { ORC_E2LSH = 0, ORC_SRP = 1 };

/* ------------------------------------------------------------------------ */
/* 1. decoding                                                               */
/* ------------------------------------------------------------------------ */

/* OCP 8-bit E4M3FN: 1 sign bit, 4 exponent bits (bias 7), 3 mantissa bits,
 * no infinities; exponent field 0 encodes subnormals m/8 * 2^-6; the pattern
 * S.1111.111 is NaN.  Value written straight from that definition. */
double orc_fp8_e4m3fn_value(uint8_t bits)
{
    int sign = (bits >> 7) & 1;
    int e = (bits >> 3) & 15;
    int mant = bits & 7;
    double v;
    if (e == 15 && mant == 7)
        return NAN;
    if (e == 0)
        v = ldexp((double)mant / 8.0, -6);
    else
        v = ldexp(1.0 + (double)mant / 8.0, e - 7);
    return sign ? -v : v;
}

/* BF16 is the upper half of an IEEE binary32 word. */
static double bf16_value(uint16_t bits)
{
    uint32_t w = (uint32_t)bits << 16;
    float f;
    memcpy(&f, &w, sizeof f);
    return (double)f;
}

/* x[i][j] = scale_i * q[i][j] in FP64 (exact: at most 24+8 significant bits). */
void orc_decode(const void *q, int dtype, const float *row_scale, int64_t n, int32_t d,
                int64_t ld, double *x)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double sc = row_scale ? (double)row_scale[i] : 1.0;
        for (int32_t j = 0; j < d; ++j) {
            double v;
            if (dtype == ORC_F32)
                v = (double)((const float *)q)[i * ld + j];
            else if (dtype == ORC_BF16)
                v = bf16_value(((const uint16_t *)q)[i * ld + j]);
            else
                v = orc_fp8_e4m3fn_value(((const uint8_t *)q)[i * ld + j]);
            x[i * (int64_t)d + j] = sc * v;
        }
    }
}

/* Storing FP32 rows in low precision (the precision path; the paper fixes no
 * storage precision).  Per row: scale = max|x| for BF16, max|x| / 448 for
 * FP8-E4M3FN (1 for a zero row), both in binary32; each stored value is the
 * binary32 quotient x / scale (FP8: clamped to [-448, 448]) rounded to the
 * nearest code, ties to the code with an even last bit.  The nearest code is
 * found by comparing the candidate values exactly in FP64. */

/* Nearest BF16 pattern: the two BF16 values around v are its binary32 bits
 * truncated to the upper half and that plus one unit in the last place. */
static uint16_t nearest_bf16(float v)
{
    uint32_t u;
    memcpy(&u, &v, sizeof u);
    uint16_t lo = (uint16_t)(u >> 16), hi = (uint16_t)(lo + 1);
    double dv = (double)v;
    double dlo = fabs(dv - bf16_value(lo)), dhi = fabs(bf16_value(hi) - dv);
    if (dlo < dhi)
        return lo;
    if (dhi < dlo)
        return hi;
    return (lo & 1) ? hi : lo;
}

/* Nearest E4M3FN pattern.  The finite non-negative codes 0x00..0x7e decode
 * to increasing values, so a bisection over their decoded values finds the
 * last code c with value(c) <= |v|; the nearer of c and c + 1 wins, a tie
 * going to the code with an even last bit.  The sign bit is that of v. */
static double g_e4m3_vals[0x7f];

static void fill_e4m3_vals(void)
{
    for (int c = 0; c <= 0x7e; ++c)
        g_e4m3_vals[c] = orc_fp8_e4m3fn_value((uint8_t)c);
}

static uint8_t nearest_e4m3fn(float v)
{
    double a = fabs((double)v);
    int lo = 0, hi = 0x7e; /* invariant: value(lo) <= a (value(0) = 0) */
    while (lo < hi) {
        int mid = (lo + hi + 1) / 2;
        if (g_e4m3_vals[mid] <= a)
            lo = mid;
        else
            hi = mid - 1;
    }
    int best = lo;
    if (lo < 0x7e) {
        double dlo = a - g_e4m3_vals[lo], dhi = g_e4m3_vals[lo + 1] - a;
        if (dhi < dlo || (dhi == dlo && (lo & 1)))
            best = lo + 1;
    }
    return (uint8_t)((signbit(v) ? 0x80 : 0) | best);
}

void orc_quantise_rows(const float *x, int64_t n, int32_t d, int dtype, void *q, float *scale)
{
    fill_e4m3_vals();
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const float *xr = x + i * (int64_t)d;
        float amax = 0.0f;
        for (int32_t j = 0; j < d; ++j)
            if (fabsf(xr[j]) > amax)
                amax = fabsf(xr[j]);
        float sc;
        if (dtype == ORC_BF16)
            sc = amax > 0.0f ? amax : 1.0f;
        else
            sc = amax > 0.0f ? amax / 448.0f : 1.0f;
        scale[i] = sc;
        for (int32_t j = 0; j < d; ++j) {
            float v = xr[j] / sc;
            if (dtype == ORC_BF16) {
                ((uint16_t *)q)[i * (int64_t)d + j] = nearest_bf16(v);
            } else {
                if (v > 448.0f)
                    v = 448.0f;
                if (v < -448.0f)
                    v = -448.0f;
                ((uint8_t *)q)[i * (int64_t)d + j] = nearest_e4m3fn(v);
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* 2. projections                                                            */
/* ------------------------------------------------------------------------ */

/* Count sketch (Definition "Count Sketch", Eq. eq_cs):
 *   CS(p)_l = sum over i with h(i) = l of s(i) * p_i.
 * Each coordinate is added to its bin in ascending i. */
void orc_cs_sketch(const double *x, int64_t n, int32_t d, const uint32_t *h, const int8_t *s,
                   int32_t m, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double *yi = y + i * (int64_t)m;
        for (int32_t l = 0; l < m; ++l)
            yi[l] = 0.0;
        for (int32_t j = 0; j < d; ++j)
            yi[h[j]] += (double)s[j] * x[i * (int64_t)d + j];
    }
}

/* Higher-order count sketch (Definition "Higher Order Count Sketch", Eq. eqhcs),
 * flattened by vec(.) as in the proof of the HCS normality theorem:
 *   j = i_1 + sum_{k>=2} i_k * prod_{t<k} d_t      (vector index of the tensor entry)
 *   l = l_1 + sum_{k>=2} l_k * prod_{t<k} m_t      (vector index of the sketch entry)
 *   HCS(p)_{l_1..l_N} = sum over (i_1..i_N) with h_k(i_k) = l_k of
 *                       s_1(i_1) ... s_N(i_N) * p_j.
 * The point is first padded with zeros up to D = prod d_k (Section 6).
 * hk/sk hold h_1..h_N (and s_1..s_N) back to back, d_k entries each. */
void orc_hcs_sketch(const double *x, int64_t n, int32_t d, int32_t N, const int32_t *dk,
                    const int32_t *mk, const uint32_t *hk, const int8_t *sk, double *y)
{
    int64_t D = 1, m = 1;
    for (int k = 0; k < N; ++k) {
        D *= dk[k];
        m *= mk[k];
    }
    int64_t mode_off[64];
    int64_t o = 0;
    for (int k = 0; k < N; ++k) {
        mode_off[k] = o;
        o += dk[k];
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double *padded = (double *)calloc((size_t)D, sizeof(double));
        for (int32_t j = 0; j < d; ++j)
            padded[j] = x[i * (int64_t)d + j];
        double *yi = y + i * m;
        for (int64_t l = 0; l < m; ++l)
            yi[l] = 0.0;
        for (int64_t j = 0; j < D; ++j) {
            /* recover (i_1, ..., i_N) from j, first mode fastest */
            int64_t rest = j, l = 0, mstride = 1;
            double sign = 1.0;
            for (int k = 0; k < N; ++k) {
                int64_t ik = rest % dk[k];
                rest /= dk[k];
                l += (int64_t)hk[mode_off[k] + ik] * mstride;
                mstride *= mk[k];
                sign *= (double)sk[mode_off[k] + ik];
            }
            yi[l] += sign * padded[j];
        }
        free(padded);
    }
}

/* Dense projection of E2LSH / SRP: y_l = <r_l, p> with r_l the l-th column of R[d][m]. */
void orc_dense_proj(const double *x, int64_t n, int32_t d, const float *R, int32_t m, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double *yi = y + i * (int64_t)m;
        for (int32_t l = 0; l < m; ++l)
            yi[l] = 0.0;
        for (int32_t j = 0; j < d; ++j) {
            double xj = x[i * (int64_t)d + j];
            const float *rj = R + (int64_t)j * m;
            for (int32_t l = 0; l < m; ++l)
                yi[l] += (double)rj[l] * xj;
        }
    }
}

/* Assignment of sketch components to tables (a reading: the paper leaves
 * open which of the m components form each of the tables).  Component l goes
 * to code position slot[l] (table slot[l] / K, rank slot[l] % K); position p
 * holds the sum of the components assigned to it, which for a permutation is
 * the component slot^-1(p) itself. */
void orc_assign_components(const double *y, int64_t n, int32_t m, const uint32_t *slot, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double *oi = out + i * (int64_t)m;
        for (int32_t p = 0; p < m; ++p)
            oi[p] = 0.0;
        for (int32_t l = 0; l < m; ++l)
            oi[slot[l]] += y[i * (int64_t)m + l];
    }
}

/* ------------------------------------------------------------------------ */
/* 3. discretisation                                                         */
/* ------------------------------------------------------------------------ */

/* E2LSH family: code_l = floor((alpha * y_l + b_l) / w).
 * near_edge[l] = 1 when v_l lies within 1e-4*w of a multiple of w (those
 * codes are the ones a different but correct rounding order may flip). */
void orc_disc_e2lsh(const double *y, int64_t n, int32_t m, const float *b, float w, double alpha,
                    int32_t *codes, uint8_t *near_edge)
{
    double ww = (double)w;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        for (int32_t l = 0; l < m; ++l) {
            double t = alpha * y[i * (int64_t)m + l];
            double v = t + (double)b[l];
            double c = floor(v / ww);
            /* codes are stored as int32; values beyond its range saturate */
            if (c < -2147483648.0)
                c = -2147483648.0;
            if (c > 2147483647.0)
                c = 2147483647.0;
            codes[i * (int64_t)m + l] = (int32_t)c;
            if (near_edge) {
                double dist = fabs(v - ww * nearbyint(v / ww));
                near_edge[i * (int64_t)m + l] = dist < 1e-4 * ww;
            }
        }
    }
}

/* SRP family: bit_l = 1 if y_l > 0 else 0.  near_edge when |y_l| < 1e-6 * ||x_i||. */
void orc_disc_srp(const double *y, const double *xnorm, int64_t n, int32_t m, int32_t *bits,
                  uint8_t *near_edge)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        for (int32_t l = 0; l < m; ++l) {
            double v = y[i * (int64_t)m + l];
            bits[i * (int64_t)m + l] = v > 0.0 ? 1 : 0;
            if (near_edge)
                near_edge[i * (int64_t)m + l] = fabs(v) < 1e-6 * xnorm[i];
        }
    }
}

void orc_row_norms(const double *x, int64_t n, int32_t d, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int32_t j = 0; j < d; ++j)
            acc += x[i * (int64_t)d + j] * x[i * (int64_t)d + j];
        out[i] = sqrt(acc);
    }
}

/* ------------------------------------------------------------------------ */
/* 4. bucket keys                                                            */
/* ------------------------------------------------------------------------ */

/* Finaliser of SplitMix64 (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014; variant 13 constants of
 * D. Stafford's mixer study): xor-shift 30, multiply, xor-shift 27, multiply,
 * xor-shift 31.  A bijection on 64-bit words. */
uint64_t orc_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * UINT64_C(0xbf58476d1ce4e5b9);
    z = (z ^ (z >> 27)) * UINT64_C(0x94d049bb133111eb);
    return z ^ (z >> 31);
}

/* Bucket key of table t for the E2LSH family: a 64-bit digest of the K-tuple
 * (c_0 .. c_{K-1}) = codes[tK .. tK+K-1].
 *   narrow tuple (every c_r in [-128, 127]): words of 8 codes, one byte each,
 *     code r in byte (r mod 8) of word floor(r/8);
 *   otherwise: words of 2 codes, 32 bits each, code r in half (r mod 2) of
 *     word floor(r/2).
 *   h = mix64(2t + wide);  for each word W: h = mix64(h xor W);  key = h.
 * Distinct tuples give distinct word sequences, and each step is a bijection
 * of the word, so keys of distinct tuples collide only by chance. */
static uint64_t e2lsh_key(const int32_t *c, int32_t K, int32_t t)
{
    int wide = 0;
    for (int32_t r = 0; r < K; ++r)
        if (c[r] < -128 || c[r] > 127)
            wide = 1;
    uint64_t h = orc_mix64(((uint64_t)t << 1) | (uint64_t)wide);
    int32_t per = wide ? 2 : 8;
    int32_t nw = (K + per - 1) / per;
    for (int32_t wi = 0; wi < nw; ++wi) {
        uint64_t W = 0;
        for (int32_t r = wi * per; r < K && r < (wi + 1) * per; ++r) {
            int pos = r - wi * per;
            if (wide)
                W |= (uint64_t)(uint32_t)c[r] << (32 * pos);
            else
                W |= (uint64_t)(uint8_t)(int8_t)c[r] << (8 * pos);
        }
        h = orc_mix64(h ^ W);
    }
    return h;
}

void orc_keys_e2lsh(const int32_t *codes, int64_t n, int32_t m, int32_t K, int32_t L,
                    uint64_t *keys)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        for (int32_t t = 0; t < L; ++t)
            keys[(int64_t)t * n + i] = e2lsh_key(codes + i * (int64_t)m + (int64_t)t * K, K, t);
}

/* SRP family: the K sign bits of table t, bit r = sgn of component tK + r. */
void orc_keys_srp(const int32_t *bits, int64_t n, int32_t m, int32_t K, int32_t L, uint64_t *keys)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        for (int32_t t = 0; t < L; ++t) {
            uint64_t k = 0;
            for (int32_t r = 0; r < K; ++r)
                if (bits[i * (int64_t)m + (int64_t)t * K + r])
                    k |= UINT64_C(1) << r;
            keys[(int64_t)t * n + i] = k;
        }
}

/* ------------------------------------------------------------------------ */
/* 5. index: per table, the points grouped by key                           */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint64_t key;
    uint32_t id;
} kv_t;

static int kv_cmp(const void *a, const void *b)
{
    const kv_t *x = (const kv_t *)a, *y = (const kv_t *)b;
    if (x->key != y->key)
        return x->key < y->key ? -1 : 1;
    return x->id < y->id ? -1 : (x->id > y->id ? 1 : 0);
}

/* Per table t: sort (key, id) pairs, id = id_base + row; then the distinct keys
 * in increasing order, ukeys[t][u], and bucket u = sorted_ids[t][offs[t][u] ..
 * offs[t][u+1]).  ukeys is [L][n], offs is [L][n+1]; nuniq[t] = number of keys. */
void orc_build_index(const uint64_t *keys, int64_t n, int32_t L, int64_t id_base,
                     uint32_t *sorted_ids, uint64_t *sorted_keys, uint64_t *ukeys, uint32_t *offs,
                     int64_t *nuniq)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t t = 0; t < L; ++t) {
        kv_t *a = (kv_t *)malloc(sizeof(kv_t) * (size_t)(n > 0 ? n : 1));
        for (int64_t i = 0; i < n; ++i) {
            a[i].key = keys[(int64_t)t * n + i];
            a[i].id = (uint32_t)(id_base + i);
        }
        qsort(a, (size_t)n, sizeof(kv_t), kv_cmp);
        int64_t u = 0;
        for (int64_t i = 0; i < n; ++i) {
            sorted_ids[(int64_t)t * n + i] = a[i].id;
            sorted_keys[(int64_t)t * n + i] = a[i].key;
            if (i == 0 || a[i].key != a[i - 1].key) {
                ukeys[(int64_t)t * n + u] = a[i].key;
                offs[(int64_t)t * (n + 1) + u] = (uint32_t)i;
                ++u;
            }
        }
        offs[(int64_t)t * (n + 1) + u] = (uint32_t)n;
        nuniq[t] = u;
        free(a);
    }
}

/* ------------------------------------------------------------------------ */
/* 6. query: union of buckets, exact re-rank                                 */
/* ------------------------------------------------------------------------ */

static int64_t find_key(const uint64_t *uk, int64_t nu, uint64_t key)
{
    int64_t lo = 0, hi = nu;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (uk[mid] < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    return (lo < nu && uk[lo] == key) ? lo : -1;
}

static int u32_cmp(const void *a, const void *b)
{
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

typedef struct {
    double score;
    int64_t id;
} sc_t;

static int sc_cmp(const void *a, const void *b)
{
    const sc_t *x = (const sc_t *)a, *y = (const sc_t *)b;
    if (x->score != y->score)
        return x->score < y->score ? -1 : 1;
    return x->id < y->id ? -1 : (x->id > y->id ? 1 : 0);
}

/* One query against nseg index segments (each built with orc_build_index over
 * its own rows; seg_n[s] points, L tables).  Candidate set = union over
 * segments and tables of the bucket holding the query's key, restricted to
 * ids < watermark.  Score: Euclidean distance (metric 0) or 1 - cos (metric 1,
 * cos = 0 when a norm is 0).  base[id][d] holds every point by global id.
 * Writes the k best (score, id) ascending, padded with (+inf, -1); returns the
 * number of distinct candidates. */
int64_t orc_query_one(int32_t nseg, const int64_t *seg_n, int32_t L,
                      const uint32_t *const *seg_sorted_ids, const uint64_t *const *seg_ukeys,
                      const uint32_t *const *seg_offs, const int64_t *const *seg_nuniq,
                      const double *base, int32_t d, const double *q, const uint64_t *qkeys,
                      int64_t qkey_ld, int32_t k, int64_t watermark, int metric,
                      int64_t *ids_out, double *score_out)
{
    int64_t cap = 0;
    for (int32_t s = 0; s < nseg; ++s)
        for (int32_t t = 0; t < L; ++t) {
            int64_t u = find_key(seg_ukeys[s] + (int64_t)t * seg_n[s], seg_nuniq[s][t],
                                 qkeys[(int64_t)t * qkey_ld]);
            if (u >= 0) {
                const uint32_t *o = seg_offs[s] + (int64_t)t * (seg_n[s] + 1);
                cap += o[u + 1] - o[u];
            }
        }
    uint32_t *c = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(cap > 0 ? cap : 1));
    int64_t nc = 0;
    for (int32_t s = 0; s < nseg; ++s)
        for (int32_t t = 0; t < L; ++t) {
            int64_t u = find_key(seg_ukeys[s] + (int64_t)t * seg_n[s], seg_nuniq[s][t],
                                 qkeys[(int64_t)t * qkey_ld]);
            if (u < 0)
                continue;
            const uint32_t *o = seg_offs[s] + (int64_t)t * (seg_n[s] + 1);
            const uint32_t *ids = seg_sorted_ids[s] + (int64_t)t * seg_n[s];
            for (uint32_t p = o[u]; p < o[u + 1]; ++p)
                if ((int64_t)ids[p] < watermark)
                    c[nc++] = ids[p];
        }
    qsort(c, (size_t)nc, sizeof(uint32_t), u32_cmp);
    int64_t nu = 0;
    for (int64_t i = 0; i < nc; ++i)
        if (i == 0 || c[i] != c[i - 1])
            c[nu++] = c[i];

    double qn = 0.0;
    for (int32_t j = 0; j < d; ++j)
        qn += q[j] * q[j];
    qn = sqrt(qn);
    sc_t *sc = (sc_t *)malloc(sizeof(sc_t) * (size_t)(nu > 0 ? nu : 1));
    for (int64_t i = 0; i < nu; ++i) {
        const double *x = base + (int64_t)c[i] * d;
        double acc = 0.0;
        if (metric == ORC_E2LSH) {
            for (int32_t j = 0; j < d; ++j) {
                double df = q[j] - x[j];
                acc += df * df;
            }
            sc[i].score = sqrt(acc);
        } else {
            double xn = 0.0;
            for (int32_t j = 0; j < d; ++j) {
                acc += q[j] * x[j];
                xn += x[j] * x[j];
            }
            xn = sqrt(xn);
            double cosv = (qn > 0.0 && xn > 0.0) ? acc / (qn * xn) : 0.0;
            sc[i].score = 1.0 - cosv;
        }
        sc[i].id = c[i];
    }
    qsort(sc, (size_t)nu, sizeof(sc_t), sc_cmp);
    for (int32_t r = 0; r < k; ++r) {
        if (r < nu) {
            ids_out[r] = sc[r].id;
            score_out[r] = sc[r].score;
        } else {
            ids_out[r] = -1;
            score_out[r] = INFINITY;
        }
    }
    free(sc);
    free(c);
    return nu;
}

/* Threads of the OpenMP loops above (for timing the oracle at a given count). */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }

int orc_max_threads(void) { return omp_get_max_threads(); }

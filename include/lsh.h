/*
 * lsh.h -- C ABI of liblsh, count-sketch LSH hashing and indexing on MI355X.
 *
 * Implements, on one gfx950 GPU, the hashcode generation and index
 * construction of Verma & Pratap, "Faster and Space Efficient Indexing for
 * Locality Sensitive Hashing":
 *   - CS-E2LSH / CS-SRP   (Section 4.1 Definition CS_Eucl_LSH, Section 5.1
 *                          Definition cs_consine_lsh): count-sketch projection
 *                          (Section 3.2 Definition def_cs, Eq. eq_cs), then
 *                          floor((sqrt(m) y + b)/w) or sgn(y);
 *   - HCS-E2LSH / HCS-SRP (Section 4.2 Definition HCS_Eucl_LSH, Eq.
 *                          eq_hca_eucl_lsh; Section 5.2 Definition
 *                          hcs_consine_lsh): higher-order count sketch of the
 *                          reshaped tensor (Definition def_hcs, Eq. eqhcs);
 *   - dense E2LSH / SRP   (Section 3.1, Eq. datar_lsh and Definition srp): the
 *                          O(md) baseline, y = x R;
 *   - the (m, tau) index  (Section 3.1): the K codes of each of L tables form a
 *                          bucket key, every point is stored in its bucket;
 *   - the query           (Section 3.1 and Section 6): union of the probed
 *                          buckets, re-ranked by exact distance, top-k.
 *
 * Conventions for every call:
 *   - All array arguments are DEVICE pointers owned by the caller unless marked
 *     "host".  The library never allocates or frees device memory; scratch
 *     space comes in through explicit workspace arguments whose size the
 *     matching *_bytes() function returns.
 *   - Work is enqueued asynchronously on `stream` (a hipStream_t; NULL = the
 *     default stream), which belongs to the current device (hipGetDevice;
 *     lsh_build_index and lsh_hash_cs_noalloc with the recheck return
 *     LSH_EINVAL otherwise, since their per-device state is the current
 *     device's), and ordered on it (lsh_build_index may also use a second
 *     stream the caller gives it, joined back to `stream`).  Nothing blocks
 *     except argument validation on the host.
 *   - Return value: LSH_OK, or a negative lsh_status with a message available
 *     from lsh_last_error() (thread-local).  On LSH_EINVAL, LSH_ENOMEM and
 *     LSH_ERANGE nothing was enqueued.  LSH_EHIP means the runtime refused a
 *     launch or copy; kernels of the same call enqueued before it may run.
 *   - n = 0 is a valid no-op wherever n appears.
 *   - Hashcode length m = K * L: one sketch of m components per point, split
 *     into L tables of K components.  By default table t owns components
 *     [tK, tK+K); lsh_disc.comp_slot assigns them to tables in another order.
 */
#ifndef LSH_H
#define LSH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LSH_OK = 0,
    LSH_EINVAL = -1, /* an argument is out of range or inconsistent */
    LSH_ENOMEM = -2, /* a workspace or index buffer is smaller than required */
    LSH_EHIP = -3,   /* the HIP runtime reported an error (message has it) */
    LSH_ERANGE = -5  /* a size exceeds what the index format can hold */
} lsh_status;

typedef enum { LSH_E2LSH = 0, LSH_SRP = 1 } lsh_family;

typedef enum {
    LSH_F32 = 0,        /* IEEE binary32 */
    LSH_BF16 = 1,       /* bfloat16 bit patterns, value = row_scale[i] * bf16 */
    LSH_FP8_E4M3FN = 2  /* OCP FP8 E4M3FN bit patterns, value = row_scale[i] * fp8 */
} lsh_dtype;

/* A set of n points of dimension d, row-major: point i, coordinate j is
 * element x[i*ld + j].  row_scale is required for LSH_BF16 / LSH_FP8_E4M3FN
 * and must be NULL for LSH_F32.  x must stay valid until the enqueued work
 * completes. */
typedef struct lsh_points {
    const void *x;
    int32_t dtype;           /* lsh_dtype */
    const float *row_scale;  /* [n] or NULL */
    int64_t n;
    int32_t d;
    int64_t ld;              /* >= d, in elements */
} lsh_points;

/* Discretisation and table layout. */
typedef struct lsh_disc {
    int32_t family;   /* lsh_family */
    int32_t m;        /* hashcode length; must equal K * L */
    int32_t K;        /* components per table, 1..64 (SRP keys hold K bits) */
    int32_t L;        /* number of tables, >= 1 */
    float w;          /* E2LSH bucket width, w > 0 (ignored for SRP) */
    const float *b;   /* [m] shifts in [0, w) (E2LSH only; NULL for SRP) */
    int32_t recheck;  /* 0: the sketch is summed exactly in fixed point (each
                         term truncated to a multiple of 2^-k, k chosen per row
                         so no bin can overflow) and discretised in FP32.  Such
                         a code differs from the FP64 evaluation only when its
                         value v = (sqrt(m) y + b) / w lies within
                         sqrt(m) * scale * (c_max + s + 1) * 2^-k / w +
                         2^-20 * (1 + |v|) of an integer (c_max: the largest bin
                         population, s: the times a long row's bins were
                         rescaled); at |v| < 128 and unit-scale rows this is
                         far below 1e-4, while huge values (|v| near 2^23 and
                         above) make every code uncertain: use recheck there.
                         counters[0] counts these components.  1: every
                         component whose value lies
                         within a rigorous bound of its error from a bin edge
                         (E2LSH) or from zero (SRP) is recomputed in FP64 in
                         ascending coordinate order, so codes equal those of an
                         FP64 evaluation.  CS/HCS only; needs d <= 32768.
                         2: as 1, with the recheck's table (the CSR of h)
                         that an earlier call with recheck = 1 built in the
                         same workspace for the same h (or h_k), d and m, in
                         stream order: the call does not build it again.
                         lsh_hash_cs_noalloc refuses 2. */
    const uint32_t *comp_slot; /* [m] device array or NULL (CS/HCS only).  Sketch
                         component l is written to code position comp_slot[l],
                         i.e. component comp_slot[l] % K of table
                         comp_slot[l] / K.  Meant to be a permutation of
                         [0, m) (a position assigned several components holds
                         their sum).  NULL: component l is position l, so table
                         t owns components [tK, tK+K).  A permutation drawn at
                         random spreads the components that share a mode index
                         of a higher-order sketch over all tables. */
} lsh_disc;

/* Outputs.  Any pointer may be NULL to skip that output. */
typedef struct lsh_out {
    uint64_t *keys;     /* [L][key_ld]: bucket key of point i in table t at keys[t*key_ld + i].
                           SRP: bit r = sign bit of component tK + r.
                           E2LSH: 64-bit digest of the K codes of the table,
                           computed as specified under "E2LSH bucket key" below. */
    int64_t key_ld;     /* 0 means n */
    int32_t *codes;     /* [n][m] E2LSH codes (int32, saturated) or SRP bits (0/1) */
    float *proj;        /* [n][m] projection y before any sqrt(m) scale, row scale applied */
    uint64_t *counters; /* [4], accumulated (not reset) by the call:
                           [0] recheck = 1: components recomputed in FP64;
                               recheck = 0 (CS/HCS): components whose FP32
                               value lies within the fast path's error
                               bound of a bin edge (E2LSH) or of zero (SRP),
                               the only ones whose code may differ from the
                               FP64 evaluation's,
                           [1] of those, components whose code changed,
                           [2] E2LSH codes that saturated to the int32 range,
                           [3] coordinates whose hash state is out of range
                               (h[j] >= m, a per-mode h_k >= m_k, or
                               comp_slot >= m); such an entry is taken as 0.
                               Zero for valid state. */
} lsh_out;

/*
 * E2LSH bucket key.  For table t with codes c_0..c_{K-1} (int32):
 *   narrow (every c_r in [-128,127]): words of 8 codes, code r is byte (r mod 8)
 *       (two's complement) of word floor(r/8);
 *   wide: words of 2 codes, code r is the 32-bit half (r mod 2) of word floor(r/2);
 *   h = F(2t + wide); for each word W in order: h = F(h XOR W); key = h;
 *   F = the SplitMix64 finaliser (Steele, Lea and Flood 2014): z ^= z>>30;
 *       z *= 0xbf58476d1ce4e5b9; z ^= z>>27; z *= 0x94d049bb133111eb; z ^= z>>31.
 */

/* ---------------------------------------------------------------- storage */

/* Store n FP32 rows x[i*ldx + j] (j < d) as low-precision codes with one FP32
 * scale per row, the form lsh_points reads with dtype LSH_BF16 or
 * LSH_FP8_E4M3FN.  The paper fixes no storage precision; this is the storage
 * of the precision path (value = row_scale[i] * decoded code).
 *   LSH_BF16:       row_scale[i] = max_j |x_ij| (1 for a zero row);
 *                   q[i*ldq + j] = bf16(x_ij / row_scale[i]) as uint16 bits.
 *   LSH_FP8_E4M3FN: row_scale[i] = max_j |x_ij| / 448 (1 for a zero row);
 *                   q[i*ldq + j] = e4m3fn(clamp(x_ij / row_scale[i], -448, 448))
 *                   as uint8 bits.
 * Each division is a binary32 division rounded to nearest even, and each
 * conversion rounds to the nearest code, ties to the even code (a negative
 * zero or a negative value that rounds to zero keeps its sign bit).
 * x, q, row_scale: device arrays owned by the caller; x must hold finite
 * values (a NaN or infinity makes its row's codes and scale unspecified).
 * EINVAL on a bad shape (d < 1, ldx < d, ldq < d) or another dtype. */
lsh_status lsh_quantize_rows(const float *x, int64_t n, int32_t d, int64_t ldx, int32_t dtype,
                             void *q, int64_t ldq, float *row_scale, void *stream);

/* ---------------------------------------------------------------- hashing */

/* Workspace bytes for lsh_hash_cs / lsh_hash_hcs (0 unless recheck is 1 or 2). */
size_t lsh_hash_workspace_bytes(int32_t d, int32_t m, int32_t recheck);

/* CS-E2LSH / CS-SRP of every point (Definitions CS_Eucl_LSH and
 * cs_consine_lsh): y_l = sum over j with h[j] = l of s[j] * x_j, then the
 * family's discretisation, codes and keys.
 *   h: [d] bins in [0, m); s: [d] signs, each +1 or -1.
 * Limits: m <= 16384, and one wave's LDS share must fit a CU's 160 KB: its
 * bins take 4 (m + m/16 + 64) bytes rounded up to a power of two, the shifts
 * 4 (m + m/16) bytes, the key seeds 16 L bytes, and the row's hash entries
 * about 4 d bytes (d rounded up to a multiple of 2048 for rows longer than
 * 1024 elements): m reaches about 8192 (short rows) and d about 38,000
 * (small m), one wave per workgroup at the limits.  EINVAL names the bytes
 * needed.  EINVAL on bad shapes, ENOMEM if ws_bytes is short. */
lsh_status lsh_hash_cs(const lsh_points *pts, const uint32_t *h, const int8_t *s,
                       const lsh_disc *disc, const lsh_out *out, void *workspace,
                       size_t ws_bytes, void *stream);

/* lsh_hash_cs for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same computation, arguments and outputs as lsh_hash_cs, without the
 * workspace.  With recheck = 1 the recheck's table (the CSR of h) is kept in
 * a static device array of 197,120 bytes per GPU, held until the process
 * ends; the call allocates and frees nothing.  Limits with recheck = 1:
 * d <= 32768 and m <= 16384, else EINVAL.  Every call on one GPU shares that
 * GPU's array and overwrites it, so calls with recheck = 1 that overlap on
 * one GPU (on different streams, or from different threads before the first
 * completes) race and give wrong codes; serialise them on one stream.  The
 * caller still owns and passes the inputs and outputs. */
lsh_status lsh_hash_cs_noalloc(const lsh_points *pts, const uint32_t *h, const int8_t *s,
                               const lsh_disc *disc, const lsh_out *out, void *stream);

/* HCS-E2LSH / HCS-SRP (Definitions HCS_Eucl_LSH and hcs_consine_lsh).  The
 * point is read as an N-order tensor d_1 x ... x_N (first mode fastest,
 * zero-padded at the end when d < prod d_k, as in Section 6) and sketched
 * with per-mode hashes h_k:[d_k] -> [m_k] and signs s_k; component
 * l = l_1 + l_2 m_1 + l_3 m_1 m_2 + ... of vec(HCS).
 *   N: 1..8; d_k, m_k: host arrays [N]; prod m_k must equal disc->m.
 *   h_k, s_k: device arrays holding h_1..h_N (s_1..s_N) back to back
 *   (sum d_k entries). */
lsh_status lsh_hash_hcs(const lsh_points *pts, int32_t N, const int32_t *d_k, const int32_t *m_k,
                        const uint32_t *h_k, const int8_t *s_k, const lsh_disc *disc,
                        const lsh_out *out, void *workspace, size_t ws_bytes, void *stream);

/* Independent tables (the protocol of Section 6: L hash tables, each built
 * from a sketch of its own with K components).  Table t has its own count
 * sketch y^t_r = sum over j with h_t(j) = r of s_t(j) x_j, r < K (Definition
 * def_cs with m = K), discretised as floor((sqrt(K) y^t_r + b[tK + r]) / w)
 * (Definition CS_Eucl_LSH at m = K) or [y^t_r > 0] (Definition
 * cs_consine_lsh); its K codes form its key as for lsh_hash_cs.  Each point
 * costs O(L d) additions against O(d) for lsh_hash_cs.
 *   h: [L][d] bins in [0, K) (table t at h[t*d + j]); s: [L][d] signs.
 *   disc: m = K * L, b[m] with table t's shifts at [tK, tK + K); comp_slot
 *   must be NULL; recheck is ignored: the sums are exact 64-bit fixed point
 *   (error below 2^-62 * d * max|x| per term) and discretised in FP64, so
 *   codes equal the FP64 evaluation except within that error of an edge.
 *   out: as for lsh_hash_cs (codes/proj at position tK + r).
 * Limits: L <= 64; the state takes about d * L bytes of LDS plus up to
 * 1024 * K + 2048 bytes per wave, at most 160 KB in all (EINVAL
 * beyond).  Any dtype. */
lsh_status lsh_hash_cs_tables(const lsh_points *pts, const uint32_t *h, const int8_t *s,
                              const lsh_disc *disc, const lsh_out *out, void *stream);

/* HCS variant of lsh_hash_cs_tables (Definitions HCS_Eucl_LSH and
 * hcs_consine_lsh with one higher-order sketch per table): table t reads the
 * point as the tensor d_1 x ... x d_N (first mode fastest, zero-padded) and
 * sketches it with its own per-mode hashes h_{t,k}: [d_k] -> [m_k] and signs.
 *   prod m_k must equal K.  h_k, s_k: [L][sum d_k], table t's N mode tables
 *   back to back at offset t * sum d_k.  Other arguments as above. */
lsh_status lsh_hash_hcs_tables(const lsh_points *pts, int32_t N, const int32_t *d_k,
                               const int32_t *m_k, const uint32_t *h_k, const int8_t *s_k,
                               const lsh_disc *disc, const lsh_out *out, void *stream);

/* Dense E2LSH / SRP (Section 3.1): y = x R on FP32 matrix cores, then
 * floor((y + b)/w) (no sqrt(m) scale) or sgn(y).  R: [d][m] row-major FP32.
 * F32 points only; recheck must be 0 and comp_slot NULL (permute the
 * columns of R instead). */
lsh_status lsh_hash_dense(const lsh_points *pts, const float *R, const lsh_disc *disc,
                          const lsh_out *out, void *stream);

/* Dense E2LSH / SRP with BF16 operands on the BF16 matrix cores (FP32
 * accumulation): the low-precision bound of the dense baseline.  Points are
 * LSH_BF16 codes with row scales; Rt holds the projection vectors as rows,
 * Rt[l*ldr + j] = r_l[j] (BF16 bits, ldr >= d), i.e. R transposed.  Then
 * y_l = row_scale[i] * sum_j q_ij r_l[j] (FP32) is discretised as in
 * lsh_hash_dense.  The FP32 sums of exact BF16 products deviate from the FP64
 * evaluation by FP32 rounding over d terms.  recheck must be 0 and comp_slot
 * NULL. */
lsh_status lsh_hash_dense_bf16(const lsh_points *pts, const uint16_t *Rt, int64_t ldr,
                               const lsh_disc *disc, const lsh_out *out, void *stream);

/* ------------------------------------------------------------------ index */

typedef struct lsh_index lsh_index; /* host-side descriptor; arrays live in caller memory */

/* Device view of a built index (Section 3.1: bucket of each key per table).
 * Table t: distinct keys ukeys[t*n + u] ascending for u < nuniq[t]; bucket u
 * holds ids sorted_ids[t*n + offs[t*(n+1) + u] .. t*n + offs[t*(n+1) + u + 1]),
 * ascending. */
typedef struct lsh_index_view {
    int64_t n;
    int32_t L;
    int64_t id_base;
    uint32_t *sorted_ids;  /* [L][n] */
    uint64_t *ukeys;       /* [L][n] (first nuniq[t] valid) */
    uint32_t *offs;        /* [L][n+1] (first nuniq[t]+1 valid) */
    int64_t *nuniq;        /* [L] */
} lsh_index_view;

/* Bytes of device memory an index over n points and L tables occupies. */
size_t lsh_index_bytes(int64_t n, int32_t L);
/* Bytes of temporary workspace lsh_build_index needs. */
size_t lsh_build_workspace_bytes(int64_t n, int32_t L);

/* Group the n points into buckets, per table (Section 3.1: every point is
 * stored in the bucket of its key in every table): the (key, id) pairs, ids =
 * id_base + i, are put in (key, id) order, then the distinct keys and bucket
 * offsets are written.  The order is built by a split on the top varying key
 * bits, sorts of the resulting segments in LDS and a pivot split of heavy
 * buckets; the result equals a stable sort of the keys.
 * keys: [L][key_ld] (key_ld 0 means n).  mem: index storage (lsh_index_bytes,
 * 256-byte aligned), ws: workspace (lsh_build_workspace_bytes, 256-byte
 * aligned; free for reuse once the enqueued work completes).  On success
 * *out receives a descriptor (release with lsh_index_free).
 * side_stream: NULL, or a second stream of the same device.  Given one
 * (other than `stream`), a build of more than 4096 points whose `stream` is
 * not capturing a graph runs its heavy-bucket split and sort there,
 * concurrently with the segment sorts, and `stream` waits for them before the
 * last kernel: the build as a whole stays ordered on `stream`, and work enqueued
 * on side_stream before the call runs before those kernels.  The fork and
 * join use a pair of events of the library per device, taken under a lock.
 * ERANGE if id_base + n exceeds 2^32 - 1. */
lsh_status lsh_build_index(const uint64_t *keys, int64_t key_ld, int64_t n, int32_t L,
                           int64_t id_base, void *mem, size_t mem_bytes, void *workspace,
                           size_t ws_bytes, lsh_index **out, void *stream, void *side_stream);

/* Fill *view with the device arrays of idx (host call, no GPU work). */
lsh_status lsh_index_get_view(const lsh_index *idx, lsh_index_view *view);

/* Release the host descriptor (device memory belongs to the caller). */
void lsh_index_free(lsh_index *idx);

/* Consistency counters of the last lsh_build_index that used `workspace`
 * (same n and L), read back with a copy on `stream` that this call waits for.
 * counts[0]: parts the big-segment sort could not queue (its stack bound);
 * counts[1]: look-back waits of the run-head pass that gave up.  Both are
 * zero by construction; a nonzero value means that build's index is wrong.
 * EINVAL for a NULL pointer or a workspace smaller than
 * lsh_build_workspace_bytes(n, L); EHIP if the copy fails. */
lsh_status lsh_build_check(const void *workspace, size_t ws_bytes, int64_t n, int32_t L,
                           uint32_t counts[2], void *stream);

/* lsh_build_check without the wait: enqueues on `stream` the copies of the
 * two counters into counts[0..1] (device memory or pinned host memory owned
 * by the caller) and returns; they are valid once the stream reaches them.
 * Meant for a server that checks each build beside its completion event.
 * For n = 0 nothing is enqueued and counts is not written (no build kernels
 * ran: both counts are zero).  EINVAL as lsh_build_check; EHIP if a copy
 * cannot be enqueued. */
lsh_status lsh_build_check_async(const void *workspace, size_t ws_bytes, int64_t n, int32_t L,
                                 uint32_t *counts, void *stream);

/* ------------------------------------------------------------------ query */

/* Answer nq queries against nseg index segments (1..16) with the same L
 * (Section 3.1: union of the buckets holding each query key; Section 6:
 * exact re-rank, top-k).
 *   base: every indexed point addressed by global id (row id of base).
 *   Q: the queries (any lsh_dtype); qkeys: [L][qkey_ld] keys of the queries,
 *      as produced by the lsh_hash_* call that built the index keys.
 *   Candidates with id >= id_watermark are ignored.
 *   metric: LSH_E2LSH = Euclidean distance, LSH_SRP = 1 - cos (cos = 0 when a
 *   norm is 0).  Output per query: ids[q*k + r] (int64, -1 pad), score[q*k + r]
 *   (FP32, +inf pad) in ascending (score, id) order; ncand[q] = number of
 *   distinct candidates (any output may be NULL except ids).  k: 1..64.
 *   workspace: NULL, or lsh_query_workspace_bytes(nq, k) bytes (256-byte
 *   aligned, any contents; calls that overlap on one workspace race).  With
 *   it, a batch of at most 1024 queries scores each query with several
 *   workgroups (up to four while they fit one per CU, else two), each
 *   leaving the top-k of its share of the candidates there for a second
 *   kernel that merges them; the answers are the same.
 *   ENOMEM if the workspace is smaller than that. */
lsh_status lsh_query(const lsh_index *const *segs, int32_t nseg, const lsh_points *base,
                     const lsh_points *Q, const uint64_t *qkeys, int64_t qkey_ld, int32_t k,
                     int64_t id_watermark, int32_t metric, int64_t *ids, float *score,
                     int32_t *ncand, void *workspace, size_t ws_bytes, void *stream);

/* Bytes of the optional lsh_query workspace for nq queries with k results
 * each: 0 when nq is 0 or above 1024 (such batches run unsplit) or k is
 * outside 1..64. */
size_t lsh_query_workspace_bytes(int64_t nq, int32_t k);

/* ------------------------------------------------------------------ misc */

/* Message for the last non-OK status returned on this thread. */
const char *lsh_last_error(void);

/* Library ABI version (major * 10000 + minor * 100 + patch). */
int32_t lsh_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LSH_H */

/*
 * csk.h — C ABI of the MI355X (gfx950) streaming Count-Sketch halo finder.
 *
 * The hot path of Ivkin et al., "Scalable Streaming Tools for Analyzing N-body
 * Simulations" (arXiv:1711.00975): every particle position becomes the key of the
 * mesh cell it lies in (Sec. 2.1), the keys are streamed into a Count Sketch of
 * d rows ("t" in the paper) by w counters ("b") with a bucket hash and a +-1 sign
 * hash per row (Sec. 2.2, Add), each distinct cell of the stream is queried for
 * the median of its d signed counters (Sec. 2.2, Estimate) and the k cells with
 * the largest estimates are returned (Sec. 2.2 UpdateHeap / Alg. 1; Sec. 3.1 item 4,
 * the threshold-filtered array of heavy cells).
 *
 * Conventions shared by every call
 *   - Data pointers marked (device) are caller-owned device memory that must stay
 *     valid until the stream reaches the call.  (host) pointers are read or written
 *     before the call returns.
 *   - `stream` is a hipStream_t passed as void* (NULL: the null stream).  Calls are
 *     asynchronous and stream-ordered unless marked "synchronizes".  A handle is
 *     not thread-safe; use one stream per handle.
 *   - Positions are float32, array-of-structures [n][3] = (x, y, z), in a periodic
 *     box of side L (Mpc/h); cells have side delta, G = round(L / delta) per side.
 *     The mesh is valid when delta, L > 0, 1 <= G <= 65535 and |L/delta - G| <=
 *     1e-6 G.  The first update or collect latches (delta, L); a different mesh on
 *     the same handle returns CSK_E_STATE until csk_reset.
 *   - Cell index along one axis: i = floor(p * G / L) on the exact values of p and L,
 *     wrapped into [0, G); key = (ix * G + iy) * G + iz (< 2^48).  A coordinate that
 *     is not finite or has |p| >= 2L puts the particle outside the domain: it is
 *     skipped and CSK_E_DOMAIN is latched (see "errors").
 *   - Row hash: simple tabulation over the six key bytes with tables drawn from
 *     SplitMix64(seed); bucket = ((h & 0x7FFFFFFF) * w) >> 31, sign = -1 if bit 31
 *     of h is set.  Counters are int32 and wrap modulo 2^32.
 *   - Errors: argument errors are returned at once and leave the handle unchanged.
 *     Conditions found by kernels (CSK_E_DOMAIN, CSK_E_CAPACITY) are latched on the
 *     device and returned by the next call that synchronizes (csk_topk,
 *     csk_get_counters, csk_check); CSK_E_CAPACITY takes precedence.  The latch is
 *     cleared when it is returned.  csk_last_error() gives the text of the last
 *     error raised on the calling thread.
 */
#ifndef CSK_H
#define CSK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct csk_sketch csk_sketch; /* opaque; owned by the library */
typedef int32_t csk_status;

#define CSK_OK            0
#define CSK_W_INCOMPLETE  1   /* fewer than k candidates passed theta            */
#define CSK_E_INVALID    (-1) /* bad argument                                      */
#define CSK_E_NOMEM      (-2) /* device allocation failed                          */
#define CSK_E_HIP        (-3) /* HIP runtime error                                 */
#define CSK_E_CAPACITY   (-4) /* candidate set overflowed: raise theta or capacity */
#define CSK_E_DOMAIN     (-5) /* some particle had a non-finite or |p| >= 2L coordinate */
#define CSK_E_STATE      (-6) /* mesh differs from the one latched on the handle   */

#define CSK_VARIANT_COUNT_SKETCH 0 /* Sec. 2.2: signed Add, median Estimate          */
#define CSK_VARIANT_COUNT_MIN    1 /* Sec. 2.2 Count-Min: Add +1, Estimate = minimum */

#define CSK_MAX_ROWS 32u
#define CSK_MAX_WIDTH (1u << 30)
#define CSK_DEFAULT_CANDIDATES (1u << 21)

/* Create a Count Sketch of d rows by w counters with hash tables drawn from `seed`
 * (Sec. 2.2: b x t counters, t bucket hashes and t sign hashes; Alg. 1
 * Initialization zeroes M).  1 <= d <= 32, 1 <= w <= 2^30.  Counters start at zero.
 * Allocates device memory on the current device; synchronizes. */
csk_status csk_sketch_init(csk_sketch **out, uint32_t d, uint32_t w, uint64_t seed);

/* As csk_sketch_init, with the variant (CSK_VARIANT_*) and the maximum number of
 * distinct candidate cells csk_collect may hold (0: CSK_DEFAULT_CANDIDATES). */
csk_status csk_sketch_init_ex(csk_sketch **out, uint32_t d, uint32_t w, uint64_t seed,
                              int32_t variant, uint64_t max_candidates);

/* As csk_sketch_init_ex, for a sketch whose items are cell keys divided by `group`
 * (1 <= group <= 2^30): the super-items of the hierarchical variant (Sec. 2.2 item 3:
 * items s_j / 1000; Alg. 3 Add(M1, s_i / 1000)).  Update and collect add and test
 * key / group; csk_collect_dictionary walks the ceil(G^3 / group) super-items; query
 * keys are super-items.  group 1 is csk_sketch_init_ex. */
csk_status csk_sketch_init_group(csk_sketch **out, uint32_t d, uint32_t w, uint64_t seed, int32_t variant,
                                 uint64_t max_candidates, uint32_t group);

/* Free the handle and all device memory it owns.  Synchronizes the device. */
csk_status csk_sketch_destroy(csk_sketch *s);

/* Add n particles to the sketch: for every in-domain particle and every row r,
 * M[r][bucket_r(key)] += sign_r(key) (Count-Min: += 1).  Sec. 2.2 Add; Alg. 1
 * "Processing the stream"; Alg. 4 Update; Sec. 3.1 stages 1-3.
 * pos (device): n x 3 float32.  n may be 0.  The result does not depend on the
 * order of particles or on how the stream is cut into calls. */
csk_status csk_sketch_update(csk_sketch *s, const float *pos, uint64_t n, double delta, double L,
                             void *stream);

/* csk_sketch_update for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, hosts that forbid hipMalloc.  The same counters
 * come out, but the token scratch is a fixed 64 MiB array that the library holds on
 * each device for the life of the process (set up by csk_sketch_init on that device),
 * so this call never allocates or frees.  A stream whose scratch need exceeds 64 MiB
 * (about 3.5e6 particles at d = 5; fewer on very wide rows) returns CSK_E_CAPACITY at
 * once, before anything is launched or latched: split it into smaller calls.  Every
 * call on one device shares that device's scratch: calls that overlap in time (on
 * different streams, or from different threads) race and must be serialised by the
 * caller.  Nothing in the scratch needs clearing between calls: each call writes the
 * counts it reads.  Arguments, errors and ordering as csk_sketch_update. */
csk_status csk_sketch_update_noalloc(csk_sketch *s, const float *pos, uint64_t n, double delta, double L,
                                     void *stream);

#define CSK_UPDATE_AUTO   0 /* LDS-binned when the rows fit it, else global atomics  */
#define CSK_UPDATE_BINNED 1 /* LDS-binned tokens, summed per counter slice          */
#define CSK_UPDATE_DIRECT 2 /* one global atomic add per row and particle           */

/* How csk_sketch_update adds to the counters; the counters come out the same either
 * way, only the speed differs (an autotuner picks per width and stream size).
 * max_wg caps the bin workgroups (0: the default).  CSK_UPDATE_BINNED on rows too wide
 * for the binned path behaves as CSK_UPDATE_AUTO. */
csk_status csk_set_update_plan(csk_sketch *s, int32_t mode, uint32_t max_wg);

#define CSK_BIN_AUTO      0 /* the sort-word kernel where it applies and is the faster, else
                               the general one */
#define CSK_BIN_GENERAL   1 /* row-interleaved hashing, bucket and sign taken apart per row */
#define CSK_BIN_SORT_WORD 2 /* tokens counting-sorted by their LDS sort words; d = 5..8,
                               w <= 2^24, a mesh that is neither grouped nor packed (else:
                               general).  The words come from packed tables when
                               w = 2^lw with lw + 1 <= floor(128 / d), else from the
                               row-interleaved tables (1024 threads, no prefetch).  For
                               csk_sketch_update_routed it selects the sort-word kernel with
                               the exclusion (row tables, two rows per pass). */

/* The tiling of the binned update (an autotuner's axes); the counters come out the same
 * for every choice.  form: CSK_BIN_*.  threads: workgroup size of the sort-word kernel,
 * 512 or 1024 (0: automatic); rows_per_pass: rows counting-sorted per LDS pass, 2 or 3
 * (0: as many as LDS holds); prefetch: 1 off, 2 on (load the next tile's positions while
 * the current one is sorted; 512 threads only), 0 automatic. */
csk_status csk_set_update_tiling(csk_sketch *s, int32_t form, uint32_t threads, uint32_t rows_per_pass,
                                 int32_t prefetch);

/* Estimates of m cell keys: est[j] = the element at index floor((d-1)/2) of the
 * ascending sort of { M[r][bucket_r(key_j)] * sign_r(key_j) } (Count-Min: the
 * minimum of M[r][bucket_r(key_j)]).  Sec. 2.2 Estimate; Alg. 4 Estimate.
 * keys (device): m uint64 (any value; only the low 48 bits are hashed).
 * est (device): m int32. */
csk_status csk_sketch_query(csk_sketch *s, const uint64_t *keys, uint64_t m, int32_t *est,
                            void *stream);

/* Cell keys of n particles (Sec. 2.1, Sec. 3.1 stage 1), for callers that want to
 * query cells of their own: keys[j] = key of particle j, or UINT64_MAX if it is
 * outside the domain (nothing is latched).  pos, keys (device). */
csk_status csk_cell_keys(const float *pos, uint64_t n, double delta, double L, uint64_t *keys,
                         void *stream);

/* Candidate pass over the particles: every in-domain particle whose cell estimate
 * is >= theta adds its cell key to the handle's set of distinct candidates (Sec. 3.1
 * item 4: keep the items above a threshold).  Repeated calls accumulate; the set
 * is emptied by csk_candidates_clear, csk_reset and csk_set_counters.  More than
 * max_candidates distinct keys latches CSK_E_CAPACITY.  pos (device). */
csk_status csk_collect(csk_sketch *s, const float *pos, uint64_t n, double delta, double L,
                       int32_t theta, void *stream);

/* The packed particle stream (Sec. 4.1: the three coordinates of a particle share 64
 * bits).  Word of a particle: qx | qy << 21 | qz << 42, q = floor(p * 2^21 / L) on the
 * exact values after the periodic wrap (the same exact floor as the cell index, on 2^21
 * cells), or UINT64_MAX when the particle is outside the domain (|p| >= 2L or not
 * finite; bit 0 of *err, device, is then set).  Its cell index on a mesh of G cells is
 * floor(q * G / 2^21), integer arithmetic, so a packed stream defines its own cells: for
 * G dividing 2^21 they are those of the float stream, otherwise a particle within L/2^21
 * of a cell boundary may move to the neighbouring cell.  pos, packed (device). */
csk_status csk_pack_positions(const float *pos, uint64_t n, double L, uint64_t *packed, uint32_t *err,
                              void *stream);
/* csk_sketch_update, csk_collect and csk_cell_keys for a packed stream (n words,
 * device), 8 bytes per particle instead of 12.  Outside-domain words are skipped and
 * latched as for float positions.  Float and packed calls may be mixed on one handle. */
csk_status csk_sketch_update_packed(csk_sketch *s, const uint64_t *packed, uint64_t n, double delta, double L,
                                   void *stream);
csk_status csk_collect_packed(csk_sketch *s, const uint64_t *packed, uint64_t n, double delta, double L,
                              int32_t theta, void *stream);
csk_status csk_cell_keys_packed(const uint64_t *packed, uint64_t n, double delta, double L, uint64_t *keys,
                                void *stream);

/* Candidate pass over the whole dictionary (Count Sketch with Full Search: Sec. 2.2
 * item 1, Alg. 1): every cell key of the G^3 mesh, G = round(L / delta), occupied or
 * not, whose estimate is >= theta is added to the candidate set; no positions are
 * read.  (delta, L) are validated and latched as in csk_collect, and the set, its
 * capacity and csk_topk behave as after csk_collect.  Asynchronous on `stream`. */
csk_status csk_collect_dictionary(csk_sketch *s, double delta, double L, int32_t theta, void *stream);

/* Hierarchical query, second layer (Count Sketch Hierarchical: Sec. 2.2 item 3, Alg. 3).
 * `coarse` is a handle made by csk_sketch_init_group with group R, whose candidate set
 * holds super-items (typically from csk_collect_dictionary with threshold theta1);
 * `fine` is an ordinary handle (group 1) updated with the same stream and mesh.  Every
 * child cell key of [j R, min((j + 1) R, G^3)) of every super-item j in coarse's set is
 * estimated from fine's counters; those with estimate >= theta join fine's candidate
 * set, from which csk_topk selects.  CSK_E_STATE unless both handles latched the same
 * mesh.  Uses coarse's candidate scratch; asynchronous on `stream`. */
csk_status csk_collect_children(csk_sketch *fine, csk_sketch *coarse, int32_t theta, void *stream);

/* Empty the candidate set. */
csk_status csk_candidates_clear(csk_sketch *s, void *stream);

/* Top-k of the candidate set: the min(k, |C|) candidates with the largest
 * estimates from the current counters, ordered by (estimate desc, key asc)
 * (Sec. 2.2 UpdateHeap; Alg. 1 query).  keys (device): k uint64; est (device):
 * k int32; *k_out (host) = the number written.  Returns CSK_W_INCOMPLETE when
 * *k_out < k and some csk_collect since the last clear used theta > INT32_MIN;
 * with theta = INT32_MIN the set is every distinct in-domain cell of the stream.
 * Synchronizes; returns a latched error if any (then *k_out is 0). */
csk_status csk_topk(csk_sketch *s, uint32_t k, uint64_t *keys, int32_t *est, uint32_t *k_out,
                    void *stream);

/* As csk_topk, without any host synchronization, so that it can be captured in a HIP
 * graph: out (device, 2 uint32) receives out[0] = the number written and out[1] = 1
 * when that is below k and the set is partial (CSK_W_INCOMPLETE of csk_topk), else 0.
 * Device-side errors stay latched for the next synchronizing call (csk_check, csk_topk,
 * csk_get_counters).  The first call with a k above every earlier one allocates
 * scratch and synchronizes: make it once before capturing. */
csk_status csk_topk_async(csk_sketch *s, uint32_t k, uint64_t *keys, int32_t *est, uint32_t *out,
                          void *stream);

/* Copy the counters out: out (device) d*w int32, row-major [d][w].  Synchronizes
 * and returns a latched error if any (the copy is made either way). */
csk_status csk_get_counters(const csk_sketch *s, int32_t *out, void *stream);

/* Replace the counters (resume from a checkpoint, or load a sum of sketches built
 * with the same d, w and seed: sketches are linear in the stream, Sec. 5).
 * in (device) d*w int32.  Empties the candidate set. */
csk_status csk_set_counters(csk_sketch *s, const int32_t *in, void *stream);

/* Zero the counters, empty the candidate set, clear the latch and the mesh. */
csk_status csk_reset(csk_sketch *s, void *stream);

/* Synchronize the stream and return (and clear) the latched device error, if any. */
csk_status csk_check(csk_sketch *s, void *stream);

/* Bytes of device memory the handle holds right now. */
uint64_t csk_device_bytes(const csk_sketch *s);

/* Text of the last error raised on the calling thread ("" if none). */
const char *csk_last_error(void);

/* ---- Batched update of many sketches ----------------------------------------------
 * Sketches of uneven size updated one after another leave most of the GPU idle when
 * they are small.  A batch shares one bin launch and one accumulate launch among up to
 * 64 sketches: each gets a fixed share of the workgroups in proportion to its largest
 * stream.  The per-sketch arithmetic is exactly that of csk_sketch_update (Sec. 2.2
 * Add; Alg. 4 Update), so each sketch ends with the counters it would have alone. */
typedef struct csk_batch csk_batch;

/* Build a batch of `count` (1..64) distinct handles with the same d (<= 8) whose
 * widths take the same hashing form (for example all powers of two up to
 * 2^(floor(128/d) - 1)).  The mesh (delta, L) is validated and latched on every
 * handle.  max_n[i] (host) bounds the particles sketch i takes per call; wg_budget is
 * the number of bin workgroups to share out (0: 512).  The handles must outlive the
 * batch.  Allocates device memory and synchronizes. */
csk_status csk_batch_create(csk_batch **out, csk_sketch *const *sketches, const uint64_t *max_n, uint32_t count,
                            double delta, double L, uint32_t wg_budget);
/* As csk_batch_create with a mesh per sketch (delta[i], L[i], host arrays): sketches of
 * different grids over the same particles (the meshes must share one cell-index path, e.g.
 * all power-of-two ratios) form one batch. */
csk_status csk_batch_create_meshes(csk_batch **out, csk_sketch *const *sketches, const uint64_t *max_n,
                                   uint32_t count, const double *delta, const double *L, uint32_t wg_budget);

/* Add n[i] particles at pos[i] (device pointers; host arrays of the batch's count) to
 * sketch i for every i, n[i] <= max_n[i].  Allocates nothing and does not synchronize,
 * so it can be captured in a HIP graph; domain errors latch on each handle.
 * Asynchronous on `stream`. */
csk_status csk_batch_update(csk_batch *b, const float *const *pos, const uint64_t *n, void *stream);

/* The top-k of every sketch of the batch (Sec. 2.2 UpdateHeap; as csk_topk_async for each
 * sketch i with k[i], keys[i], est[i], out[i], all host arrays of the batch's count holding
 * device pointers) in one set of launches.  out[i][0] = how many, out[i][1] = 1 when fewer
 * than k[i] came from a partial candidate set.  The first call, and a call after a
 * sketch's selection scratch grew, allocates and synchronizes; later calls allocate
 * nothing and do not synchronize, so they can be captured in a HIP graph. */
csk_status csk_batch_topk(csk_batch *b, const uint32_t *k, uint64_t *const *keys, int32_t *const *est,
                          uint32_t *const *out, void *stream);

/* Free the batch (the handles stay). */
/* Every sketch of the batch back to zero counters and an empty candidate set, as
 * csk_reset on each, in one launch.  Asynchronous on `stream`. */
csk_status csk_batch_reset(csk_batch *b, void *stream);

/* The candidate pass of every sketch of the batch (csk_collect on each: pos[i] (device),
 * n[i] particles, theta[i], on the mesh the sketch was batched with) as one set of
 * launches: the filter and hot-set clears and builds of every sketch whose theta is > 0,
 * then one collect launch whose workgroups are shared among the sketches in proportion
 * to their max_n.  Sec. 3.1 item 4 per sketch; results as csk_collect one by one.
 * Asynchronous; nothing is allocated, so it can be captured in a HIP graph. */
csk_status csk_batch_collect(csk_batch *b, const float *const *pos, const uint64_t *n, const int32_t *theta,
                             void *stream);

csk_status csk_batch_destroy(csk_batch *b);

/* ---- Learned router --------------------------------------------------------------
 * A small model decides which coarse cells are counted exactly: cells it predicts to
 * hold heavy cells go to an exact device hash table, every other particle to a Count
 * Sketch whose width gives the pair the memory of a plain sketch.  The features of a
 * coarse cell are the counts of a 1 % sample of the stream in it and its 26 neighbours. */

/* Add, for each particle index0 + i (i < n) in the sample, 1 to counts[coarse key]
 * (device, G_c^3 uint32, G_c = round(L / delta_c)).  Particle g is in the sample when
 * word g of the Philox4x32-10 stream 4 under key (seed mod 2^32, seed / 2^32) -- word
 * g mod 4 at counter (g / 4 mod 2^32, g / 4 / 2^32, 4, 0) -- is below `threshold`
 * (1 %: 42949672).  Out-of-domain
 * particles are skipped.  pos (device).  bitmap (device, ceil(G_c^3 / 32) words, or NULL):
 * a cell's bit (word key / 32, bit key mod 32) is set when its count leaves 0, so that
 * csk_cell_list and csk_cells_clear touch only the sampled cells. */
csk_status csk_sample_counts(const float *pos, uint64_t n, uint64_t index0, double delta_c, double L, uint64_t seed,
                             uint32_t threshold, uint32_t *counts, uint32_t *bitmap, void *stream);

/* feat[j][q] = log1pf(counts[neighbour q of cells[j]]) for q < 27: the coarse cell and its
 * 26 periodic neighbours in (dx, dy, dz) lexicographic order over {-1, 0, 1}^3;
 * feat[j][27..31] = 0.  counts, cells, feat (device); feat is m x 32 float32. */
csk_status csk_cell_features(const uint32_t *counts, double delta_c, double L, const uint64_t *cells, uint64_t m,
                             float *feat, void *stream);

/* The router's model: 27 -> 64 -> 64 -> 1 (inputs padded to 32), ReLU, fp32 master weights
 * used as bf16 operands of v_mfma_f32_16x16x16_bf16 with fp32 accumulation; output layer
 * on bf16-rounded operands with fp32 sums.  Weights He-uniform from SplitMix64(seed),
 * biases 0.  max_batch bounds a training batch and the forward chunk. */
typedef struct csk_mlp csk_mlp;
csk_status csk_mlp_create(csk_mlp **out, uint64_t seed, uint32_t max_batch);
csk_status csk_mlp_destroy(csk_mlp *m);
/* Copy the 6337 fp32 master parameters out to `out` (host), and/or load them from `in`
 * (host; resets the optimizer).  Layout: W1[64][32], b1[64], W2[64][64], b2[64], w3[64],
 * b3.  Synchronizes. */
csk_status csk_mlp_params(csk_mlp *m, float *out, const float *in);
/* Copy the gradients of the last training step (same layout) to `out` (host).  Synchronizes. */
csk_status csk_mlp_grads(csk_mlp *m, float *out);
/* logits[j] (device) of the n feature rows x (device, n x 32). */
csk_status csk_mlp_forward(csk_mlp *m, const float *x, uint64_t n, float *logits, void *stream);
/* One Adam step (lr, beta1 0.9, beta2 0.999, eps 1e-8) on the mean binary cross-entropy of
 * n <= max_batch rows x with labels y (device, 0 or 1); *loss (device, may be NULL) gets
 * the loss before the step. */
csk_status csk_mlp_train_step(csk_mlp *m, const float *x, const float *y, uint32_t n, float lr, float *loss,
                              void *stream);

/* The router's matrix product: C(i, j) = beta C(i, j) + sum_k A(i, k) B(k, j) for i < M,
 * j < N, with A(i, k) = A[i sai + k sak], B(k, j) = B[k sbk + j sbj], C(i, j) =
 * C[i sci + j scj] (device float32, any strides, so transposed operands need no copy).
 * Operands are rounded to bf16 (nearest even) and the products summed in float32 on the
 * matrix cores; beta = 0 ignores C's old contents.  M, N <= 2^20; K >= 0. */
csk_status csk_gemm_bf16(uint32_t M, uint32_t N, uint32_t K, const float *A, uint64_t sai, uint64_t sak,
                         const float *B, uint64_t sbk, uint64_t sbj, float *C, uint64_t sci, uint64_t scj,
                         float beta, void *stream);

/* Route a stream: an in-domain particle whose coarse parent (cell index / factor on each
 * axis) is in `admitted` (device, na <= 512 coarse keys of the mesh G / factor, sorted
 * ascending) adds 1 to its cell key's count in the exact table (device, table_slots a power
 * of two, keys all-ones when empty, linear probing from a fixed hash); every other
 * in-domain particle is appended, in stream order, to rest_pos (device) after the
 * *rest_count (device) particles already there, and *rest_count grows by their number
 * (rest_pos needs room for *rest_count + n).  na * factor^3 <= min(2^15, table_slots / 2),
 * so the table never fills.  Out-of-domain particles set bit 0 of *err (device).
 * workspace: device scratch of csk_route_split_workspace bytes, not shared between calls
 * in flight. */
csk_status csk_route_split_workspace(uint32_t na, uint32_t factor, uint64_t *bytes);
csk_status csk_route_split(const float *pos, uint64_t n, double delta, double L, uint32_t factor,
                           const uint64_t *admitted, uint32_t na, uint64_t *table_keys, uint32_t *table_counts,
                           uint32_t table_slots, float *rest_pos, uint64_t *rest_count, uint32_t *err,
                           void *workspace, uint64_t workspace_bytes, void *stream);

/* Exact cell counts: every in-domain particle adds 1 to its cell key's count in the table
 * (device; table_slots a power of two <= 2^31; keys all-ones and counts 0 when empty, as
 * for csk_route_split).  This is the exact histogram that the sketch approximates (the
 * router's training labels and the recall reference); n < 2^31 keeps every count below
 * 2^31.  Out-of-domain particles set bit 0 of *err (device), a key finding no free slot
 * sets bit 1 (size the table at twice the distinct cells or more). */
csk_status csk_exact_counts(const float *pos, uint64_t n, double delta, double L, uint64_t *table_keys,
                            uint32_t *table_counts, uint32_t table_slots, uint32_t *err, void *stream);

/* The k heaviest keys of an exact table (as filled by csk_exact_counts or csk_route_split),
 * ordered by (count desc, key asc), into keys / counts (device); *k_out (host) = how many,
 * min(k, keys in the table).  k <= 2^22.  Allocates scratch and synchronizes. */
csk_status csk_table_topk(const uint64_t *table_keys, const uint32_t *table_counts, uint32_t table_slots, uint32_t k,
                          uint64_t *keys, uint32_t *counts, uint32_t *k_out, void *stream);

/* The cells j < ncells with counts[j] >= min_count (device), in ascending order, into
 * cells (device, the first cap of them); *total (host) = how many there are.  Lists the
 * coarse cells the router scores.  With the bitmap of csk_sample_counts (device, or NULL)
 * only the cells whose bit is set are examined (every cell with a nonzero count has
 * one).  Allocates scratch and synchronizes. */
csk_status csk_cell_list(const uint32_t *counts, uint64_t ncells, uint32_t min_count, const uint32_t *bitmap,
                         uint64_t *cells, uint64_t cap, uint64_t *total, void *stream);
/* Zero counts[j] for every cell j whose bit is set, then the bitmap (both device): the
 * state of csk_sample_counts back to empty without writing all G_c^3 counters. */
csk_status csk_cells_clear(uint32_t *counts, uint32_t *bitmap, uint64_t ncells, void *stream);

/* Router training labels: labels[j] (device float) = 1 if coarse cell cells[j] (mesh
 * G / factor) is the coarse parent of one of the nk <= 2^17 fine keys (device, mesh of
 * delta, L), else 0.  Allocates scratch and synchronizes. */
csk_status csk_cell_labels(const uint64_t *cells, uint64_t m, const uint64_t *fine_keys, uint32_t nk, double delta,
                           double L, uint32_t factor, float *labels, void *stream);

/* Admission: of the m < 2^31 distinct cells (device keys below 2^48) with their logits
 * (device float, finite), the min(A, m) highest by (logit desc, key asc) into admitted
 * (device), in ascending key order as csk_route_split takes them; *na (host) = how many.
 * A <= 2^16.  Allocates scratch and synchronizes. */
csk_status csk_route_admit(const uint64_t *cells, const float *logits, uint64_t m, uint32_t A, uint64_t *admitted,
                           uint32_t *na, void *stream);

/* As csk_topk for a sketch of the routed rest: every key of the exact table joins the
 * candidates, and a candidate found in the table takes its exact count as its estimate.
 * Synchronizes. */
csk_status csk_topk_with_table(csk_sketch *s, const uint64_t *table_keys, const uint32_t *table_counts,
                               uint32_t table_slots, uint32_t k, uint64_t *keys, int32_t *est, uint32_t *k_out,
                               void *stream);

/* ---- The routed step without host synchronization (Sec. 2.2 Add and Estimate on the rest;
 * the learned router around them).  Every call below only enqueues work on `stream`:
 * counts stay on the device, nothing is allocated, so that the whole step -- sample,
 * listing, scoring, admission, routed update, candidate pass, merged top-k -- can be
 * captured in a HIP graph once each handle has run it eagerly.  Workspaces are device
 * scratch of the stated size, not shared between calls in flight. */

/* As csk_cell_list with *total (device uint64) instead of a host count.  workspace: at
 * least csk_cell_list_workspace(ncells) bytes. */
csk_status csk_cell_list_workspace(uint64_t ncells, uint64_t *bytes);
csk_status csk_cell_list_async(const uint32_t *counts, uint64_t ncells, uint32_t min_count, const uint32_t *bitmap,
                               uint64_t *cells, uint64_t cap, uint64_t *total, void *workspace,
                               uint64_t workspace_bytes, void *stream);

/* Logits (device float) of the coarse cells cells[0 .. min(*m, cap)) (m: device uint64):
 * the features of csk_cell_features fed through the model's fp32 master parameters with
 * every product and sum in fp32 (no bf16 rounding), all in one kernel. */
csk_status csk_route_score(csk_mlp *m, const uint32_t *counts, double delta_c, double L, const uint64_t *cells,
                           const uint64_t *m_dev, uint64_t cap, float *logits, void *stream);

/* As csk_route_admit over the first min(*m, cap) cells (m: device uint64; cap < 2^31,
 * 1 <= A <= 2^16): the admitted keys in ascending order into admitted (device, room for
 * A) and their number into *na (device uint32). */
csk_status csk_route_admit_workspace(uint64_t cap, uint32_t A, uint64_t *bytes);
csk_status csk_route_admit_async(const uint64_t *cells, const float *logits, const uint64_t *m, uint64_t cap,
                                 uint32_t A, uint64_t *admitted, uint32_t *na, void *workspace,
                                 uint64_t workspace_bytes, void *stream);

/* csk_route_split fused into the rest sketch's update: every in-domain particle whose
 * coarse parent (fine index / factor per axis) is one of admitted[0 .. *na) (device;
 * *na device uint32) adds 1 to its fine key's count in the exact table (cleared by the
 * caller: keys all-ones, counts 0), and every other one is added to s (Sec. 2.2 Add) --
 * the counters and the table of csk_route_split followed by csk_sketch_update of the
 * rest, with no rest stream written.  The sketch must count single cells (group 1);
 * factor divides G.  At most na_max = min(512, 2^15 / factor^3, table_slots / 2 /
 * factor^3) admitted cells are used: a larger *na sets bit 2 of *err (device), a full
 * table bit 1.  Domain errors latch on s as for csk_sketch_update.  workspace: at least
 * csk_route_update_workspace(factor, table_slots) bytes.  The candidate pass of the rest
 * sketch may then run over the whole stream: an admitted key reaches the top-k with its
 * exact count whatever its estimate (csk_topk_with_table).  The bin kernel follows the
 * handle's csk_set_update_tiling form (d = 5): the general kernel unless CSK_BIN_SORT_WORD
 * asks for the sort-word one; the counters are the same. */
csk_status csk_route_update_workspace(uint32_t factor, uint32_t table_slots, uint64_t *bytes);
csk_status csk_sketch_update_routed(csk_sketch *s, const float *pos, uint64_t n, double delta, double L,
                                    uint32_t factor, const uint64_t *admitted, const uint32_t *na,
                                    uint64_t *table_keys, uint32_t *table_counts, uint32_t table_slots, uint32_t *err,
                                    void *workspace, uint64_t workspace_bytes, void *stream);

/* As csk_topk_with_table with out (device, 2 uint32) in place of k_out, as csk_topk_async
 * (the first call with a larger k allocates and synchronizes). */
csk_status csk_topk_with_table_async(csk_sketch *s, const uint64_t *table_keys, const uint32_t *table_counts,
                                     uint32_t table_slots, uint32_t k, uint64_t *keys, int32_t *est, uint32_t *out,
                                     void *stream);

#ifdef __cplusplus
}
#endif

#endif /* CSK_H */

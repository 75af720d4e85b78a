/*
 * pipnn.h -- C ABI of the MI355X (gfx950) PiPNN leaf hot path.
 *
 * PiPNN ("PiPNN: Ultra-Scalable Graph-Based Nearest Neighbor Indexing",
 * arXiv 2602.21247) builds a graph index in four steps (Alg. 4):
 *   1. Partition: randomized ball carving with fanout into overlapping
 *      leaves of at most C_max points (Sec. 4.1, Alg. 5);
 *   2. Pick: per leaf, an all-pairs distance matrix computed as a dense
 *      GEMM and each row's k nearest co-members, bi-directed (Sec. 4.2);
 *   3. Prune_And_Add_Edges: those edges stream into HashPrune, a bounded
 *      per-point reservoir with one slot per LSH bucket (Sec. 3, Alg. 3);
 *   4. PruneNode: a final RobustPrune of every reservoir (Sec. 4.3, Alg. 2).
 * Queries use BeamSearch (Alg. 1).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Status: every call returns pipnn_status; 0 is success, negative values
 *    are errors. pipnn_last_error() returns a thread-local message for the
 *    last failing call on the calling thread. No C++ exception crosses this
 *    interface and no call aborts the process.
 *  - Streams: device work is enqueued on the caller's hipStream_t (0 = the
 *    null stream) and is asynchronous unless the call is marked "sync".
 *    Device faults surface as PIPNN_EDEVICE at the next synchronising call.
 *  - Pointers: arguments named d_* are device pointers; h_* are host
 *    pointers. All of them are owned by the caller and must stay valid until
 *    the enqueued work has finished. X (and H) must outlive the index.
 *  - Memory: an index created over a caller's workspace (pipnn_create's
 *    d_workspace, of at least pipnn_workspace_bytes) allocates no device
 *    memory: every device buffer it uses (sketches, norms, copies of X,
 *    partition levels, picks, candidate bins, search scratch) is a fixed
 *    slice of that workspace, and a call whose data would exceed its slice
 *    fails with PIPNN_ENOMEM. With no workspace the index allocates its
 *    buffers itself (hipMalloc, grown on demand, freed by pipnn_destroy);
 *    only such an index can grow its capacity (pipnn_reserve) for
 *    pipnn_insert. pipnn_hashprune_insert_static uses neither (see there).
 *  - Ids are uint32 point indices 0..n-1; 0xFFFFFFFF marks an empty slot.
 *  - Distances are squared L2 (metric 0) or the negated inner product
 *    (metric 1), so that smaller is always nearer (Preliminaries).
 *  - Ties are broken by (distance, id) everywhere.
 *
 * Thread safety: calls on different indices may run concurrently; calls on
 * one index must be serialised by the caller.
 */
#ifndef PIPNN_H
#define PIPNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *pipnn_stream_t; /* the same type as hipStream_t */
typedef struct pipnn_index pipnn_index;
typedef int32_t pipnn_status;

#define PIPNN_OK 0
#define PIPNN_EINVAL (-1)    /* an argument is out of range */
#define PIPNN_ENOMEM (-2)    /* a device allocation failed */
#define PIPNN_EOVERFLOW (-3) /* an output capacity is too small; the need is written back */
#define PIPNN_EDEVICE (-4)   /* a HIP runtime error, or an id >= n found on the device */
#define PIPNN_ESTATE (-5)    /* the call is not valid in the index's current state */

#define PIPNN_METRIC_L2 0 /* squared Euclidean distance */
#define PIPNN_METRIC_IP 1 /* negative inner product (MIPS) */

#define PIPNN_DTYPE_F32 0
#define PIPNN_DTYPE_F16 1
#define PIPNN_DTYPE_BF16 2

#define PIPNN_PREC_FP32 0    /* leaf GEMM on FP32 MFMA */
#define PIPNN_PREC_BF16 1    /* BF16 MFMA, FP32 accumulation */
#define PIPNN_PREC_FP8 2     /* OCP e4m3 MFMA with per-point scales, FP32 accumulation */
#define PIPNN_PREC_FP16 3    /* FP16 MFMA, FP32 accumulation */

#define PIPNN_PICKER_KNN 0        /* bi-directed k nearest co-members (Sec. 4.2) */
#define PIPNN_PICKER_ALL_TO_ALL 1 /* RobustPrune over the whole leaf (Supplement) */

#define PIPNN_EMPTY_ID 0xFFFFFFFFu

/* Hyper-parameter bundle BP of Alg. 4.
 *  metric       PIPNN_METRIC_*.
 *  c_max        C_max, the largest leaf (Sec. 4.1 keeps it small, about 1-2 thousand).
 *  c_min        C_min: buckets below it are merged (Sec. 4.1, Merge).
 *  leader_div   P_samp = 1/leader_div: a subproblem P gets
 *               l = min(leader_cap, max(2, ceil(|P|/leader_div)), |P|) leaders.
 *  leader_cap   the hard cap on leaders per subproblem (typically 1000).
 *  fanout[4]    fanout(depth) for depth 0,1,2 and >= 3 (Alg. 5); each
 *               point joins its min(fanout, l) nearest leaders' buckets.
 *               fanout[3] must be 1 so that the instance count stays bounded.
 *  k            leaf pick: each point's k nearest co-members (Sec. 4.2).
 *  hash_bits    m, hyperplanes per hash, 1..16 (Sec. 3; 12 by default).
 *  l_max        HashPrune reservoir slots per point (Alg. 3), 1..256.
 *  R            final degree bound of RobustPrune (Alg. 2), 1..256.
 *  alpha        RobustPrune's alpha (Alg. 2), >= 1, applied to the
 *               distances above (squared L2 or negated inner product).
 *  gemm_prec    PIPNN_PREC_*: arithmetic of the leaf distance GEMM. BF16,
 *               FP16 and FP8 multiply a copy of X in that format (made by
 *               pipnn_create / pipnn_prepare, d <= 768) and accumulate in
 *               FP32; FP32 needs d <= 256. When every value of X survives
 *               the encoding (the copy holds X exactly, as bf16 does for
 *               integers of up to 8 significant bits), the partition's
 *               distances and RobustPrune's rows are read from the copy
 *               too (half the bytes; the same values); otherwise the
 *               partition uses the float32 vectors for d <= 256 and the
 *               copy above. A float32 index of at most 128 dimensions
 *               keeps an fp16 copy while X passes the integer check (see
 *               pipnn_stats.data_int_exact); where that copy holds X
 *               exactly, the partition and RobustPrune read it the same
 *               way (every distance form is then the same integer in
 *               either format) and the leaf GEMM stays FP32. An L2 index of
 *               at most 128 dimensions whose values are integers spanning at
 *               most 256 consecutive values (any precision) also keeps int8
 *               rows x - lo - 128; RobustPrune then reads those (a quarter of
 *               the float32 bytes; exact integer distances, see
 *               pipnn_stats.rp_row_bits).
 *  rescore_mult 0, or r >= 2: select the r*k nearest by the GEMM distance
 *               and keep the k nearest by an FP32 direct-difference rescore.
 *  rescore_extra 0, or e >= 1 (k + e <= 32; rescore_mult then 0): select
 *               the k + e nearest by the GEMM distance, i.e. the k winners and
 *               the e just past the boundary, and keep the k nearest of them
 *               by the same rescore. A smaller margin than r*k: the selection
 *               keeps shorter lists (its cost grows with their length) and
 *               recovers a true neighbour only if the GEMM error moved it at
 *               most e places.
 *  leaf_picker  PIPNN_PICKER_*: how a leaf member picks its candidates
 *               (Sec. 4.2 and the Supplement, "Picking within Leaves"):
 *               KNN, its k nearest co-members, bi-directed (both records
 *               of each pick go to HashPrune); ALL_TO_ALL, RobustPrune
 *               (Alg. 2, lazy form) of the member over every other member
 *               of its leaf with this alpha, up to k admitted, each giving
 *               the member one record (leaves of at most 2,048 members;
 *               no rescoring; no planned / captured builds, no insertion).
 *  seed         root key of the leader sampling (Alg. 5, SampleLeaders).
 */
typedef struct {
  int32_t metric;
  int32_t c_max, c_min, leader_div, leader_cap;
  int32_t fanout[4];
  int32_t k, hash_bits, l_max, R;
  float alpha;
  int32_t gemm_prec;
  int32_t rescore_mult;
  int32_t leaf_picker;
  int32_t rescore_extra;
  uint64_t seed;
} pipnn_params;

/* Library version string. Never fails. */
const char *pipnn_version(void);

/* Message of the last failing call on this thread ("" if none). */
const char *pipnn_last_error(void);

/* Fills *p with the defaults: L2, C_max 1024, C_min 64, leader_div 200,
 * leader_cap 1000, fanout {2,1,1,1}, k 16, m 12, l_max 64, R 32, alpha 1.2,
 * FP32 GEMM, no rescore, seed 0. */
void pipnn_default_params(pipnn_params *p);

/* Bytes of the workspace an index over n points of dimension d with X of
 * x_dtype needs when a build bins at most max_batch_records candidate
 * records at a time (a leaf pick gives two records per pick: the batch is
 * max_batch_records / (2k) leaf rows, at least 65535 -- the largest leaf --
 * and at most a whole build; 0 = a whole build in one batch). The value is
 * the sum of the index's fixed buffer slices, each sized for the worst case
 * the parameters allow: a partition of the n points (Alg. 5, at most n times
 * fanout[0] * fanout[1] * fanout[2] leaf members), one batch of picks and
 * records, RobustPrune's order, search and k-NN-graph batches. pipnn_create
 * succeeds with exactly this many bytes and fails with PIPNN_ENOMEM with
 * fewer than the value for the smallest batch. Returns 0 for invalid
 * parameters, n, d or dtype. */
size_t pipnn_workspace_bytes(const pipnn_params *p, int64_t n, int32_t d, int32_t x_dtype,
                             int64_t max_batch_records);

/* Create an index over d_X (n x d, row-major, x_dtype) with hyperplanes
 * d_H (hash_bits x d, float32, row-major; Sec. 3: m random hyperplanes,
 * each given by its normal vector). Computes the per-point sketches Sketch(v)_b = H_b . v
 * (Sec. 3, Implementation) and squared norms on the stream. d_X and d_H are
 * referenced, not copied, and must outlive the index.
 * EINVAL if n < 2, d < 1, hash_bits not in 1..16, k < 1, l_max not in
 * 1..256, R not in 1..256, alpha < 1, c_max < 2, c_min > c_max, leader_div
 * < 1, leader_cap < 2, a fanout < 1, fanout[3] != 1, an unknown dtype or
 * precision, n >= 2^32 - 1, d > 256 with gemm_prec FP32, or d > 768. With a
 * reduced gemm_prec it also encodes the GEMM operand (see
 * pipnn_get_operand).
 * d_workspace / ws_bytes: a device buffer owned by the caller (256-byte
 * aligned; it must outlive the index) from which every device buffer of the
 * index is carved; the index then allocates nothing. Build batches take the
 * most leaf rows whose layout fits ws_bytes (see pipnn_workspace_bytes;
 * pipnn_get_stats reports the layout and batch). On a workspace a float32 X
 * must be 16-byte aligned (EINVAL otherwise), the point count is fixed at n,
 * and a call whose data exceed the layout (leaves with more members than
 * the bound, a knn_block of more rows than a batch) fails with ENOMEM.
 * ENOMEM if ws_bytes is below pipnn_workspace_bytes for the smallest batch
 * (this check takes no device call). NULL / 0: the index allocates its own
 * buffers (ENOMEM if that fails). */
pipnn_status pipnn_create(const pipnn_params *p, const void *d_X, int64_t n, int32_t d,
                          int32_t x_dtype, const float *d_H, void *d_workspace, size_t ws_bytes,
                          pipnn_stream_t stream, pipnn_index **out);

/* Release the index and the device buffers it allocated (none on a
 * workspace, which the caller frees afterwards). The caller must have
 * finished the work that uses the index on every stream; no device-wide
 * synchronisation is made. */
void pipnn_destroy(pipnn_index *idx);

/* (sync) Randomized ball carving (Alg. 5) of all n points into leaves of at
 * most C_max points. Leaves are returned as CSR: d_leaf_offsets[0..L]
 * (int64, offsets[0] = 0) and d_leaf_members (uint32, ascending ids within a
 * leaf). The leaf order is unspecified; leaf contents are deterministic for
 * a seed. Reads bucket sizes back to the host once per recursion level.
 * EOVERFLOW if L > cap_leaves or the member count > cap_members; the needed
 * sizes are written to *h_n_leaves and *h_n_members either way. */
pipnn_status pipnn_partition(pipnn_index *idx, int64_t *d_leaf_offsets, int64_t cap_leaves,
                             uint32_t *d_leaf_members, int64_t cap_members, int64_t *h_n_leaves,
                             int64_t *h_n_members, pipnn_stream_t stream);

/* (sync) An independent replica of the partition (the paper's replication:
 * another ball carving of the same points with other random leaders):
 * pipnn_partition with the root key of replica r -- the seed for r = 0,
 * else the first splitmix64 output from seed xor r * 0xD1B54A32D192ED03.
 * pipnn_build_leaves on each replica's leaves into the same reservoirs
 * builds the replicated index (HashPrune is order-free). EINVAL if r < 0;
 * otherwise as pipnn_partition. */
pipnn_status pipnn_partition_replica(pipnn_index *idx, int32_t replica, int64_t *d_leaf_offsets,
                                     int64_t cap_leaves, uint32_t *d_leaf_members,
                                     int64_t cap_members, int64_t *h_n_leaves,
                                     int64_t *h_n_members, pipnn_stream_t stream);

/* (sync) Plan the leaves of a later pipnn_build_leaves call: reads the
 * offsets, checks the member ids, builds the leaf kernel's work lists on the
 * device and reserves every scratch buffer of the build. pipnn_build_leaves
 * with the same d_leaf_offsets, d_leaf_members and n_leaves pointers and
 * count (and the same leaf configuration) then does no host work, reads
 * nothing back and allocates nothing, so it may be captured in a HIP graph
 * and replayed; the caller must not change the offsets or members between
 * plan and replay (ids are checked here, not again). The plan is replaced
 * by the next call. ESTATE under stream capture. */
pipnn_status pipnn_plan_leaves(pipnn_index *idx, const int64_t *d_leaf_offsets,
                               const uint32_t *d_leaf_members, int64_t n_leaves,
                               pipnn_stream_t stream);

/* Leaf-kernel layouts. PAIR: a row's operand is split over two lanes
 * (32x32 MFMA tiles, a wave owns 32 rows; operands of up to 256
 * dimensions). QUAD: over four lanes (16x16 MFMA tiles, a wave owns 16 rows,
 * half the registers per row, so more waves share a compute unit; every
 * width but the 96-dimension e4m3 operand, and the only layout above 256
 * dimensions). */
#define PIPNN_LAYOUT_PAIR 0
#define PIPNN_LAYOUT_QUAD 1

/* Leaf-kernel configuration of the index: layout (above); rows_per_item
 * 128 (PAIR: four waves of 32 rows; QUAD: eight waves of 16) or 64 (PAIR
 * only, built for operands of 65..128 dimensions); persistent 0 (one
 * workgroup per work item, dealt to the XCDs by the host) or 1 (resident
 * workgroups take the items of their XCD from a device counter, which
 * balances uneven leaves at run time). rows_per_item and persistent do not
 * change results. The two layouts sum the GEMM's products in different
 * orders, so where that arithmetic rounds (non-integer data) GEMM distances
 * can differ in the last bits between them, and with them the choice among
 * near-tied candidates; the FP32 recomputed distances of a pair do not
 * depend on the layout. The index starts with QUAD, 128 rows, static for
 * float32, bf16 and fp16 GEMM operands and PAIR, 128 rows, static for e4m3
 * (QUAD where the other is not built). EINVAL for other values or a shape
 * that is not built. */
pipnn_status pipnn_set_leaf_config(pipnn_index *idx, int32_t rows_per_item, int32_t persistent,
                                   int32_t layout);

typedef struct {
  int32_t rows_per_item, persistent, layout;
  float ms; /* best of the timed runs of the leaf pick on the sample */
} pipnn_tune_result;

/* (sync) Autotuner of the leaf kernel: times the leaf pick (distance GEMM +
 * selection, no HashPrune) on the given leaves (the first 2^25 rows' worth)
 * for every configuration pipnn_set_leaf_config accepts on this index, sets
 * the fastest, and reports each configuration's time in h_results (up to
 * cap_results; *h_n_results receives the count). */
pipnn_status pipnn_autotune(pipnn_index *idx, const int64_t *d_leaf_offsets,
                            const uint32_t *d_leaf_members, int64_t n_leaves,
                            pipnn_tune_result *h_results, int32_t cap_results,
                            int32_t *h_n_results, pipnn_stream_t stream);

/* ---- serving: growing an index in place ---- */

/* (sync) Make room for n_cap points: grows the index's per-point buffers
 * (norms, sketches, float32 copy, GEMM operand) keeping their contents, and
 * sizes the point-indexed scratch of insertion for n_cap, so that
 * insertions up to the capacity reallocate none of it. d_X (may be NULL:
 * keep the current one) rebinds the index to a new X of the same dtype and
 * dimension whose first n rows hold the current points -- the way to grow
 * past the rows of the X bound at pipnn_create: the caller allocates a
 * larger X, copies the rows, calls this, and then frees the old X (this
 * call synchronises the stream before rebinding; work on other streams that
 * reads the old X must have finished). The bound X must have n_cap rows,
 * and the caller sizes its reservoirs (n_cap x l_max), graph (n_cap x R)
 * and degree (n_cap) buffers the same way. EINVAL if n_cap >= 2^32 - 1, or
 * if a new float32 X that the leaf kernel reads directly is not 16-byte
 * aligned; ESTATE if the index was created over a workspace and n_cap
 * exceeds its point count (such an index has a fixed capacity). */
pipnn_status pipnn_reserve(pipnn_index *idx, int64_t n_cap, const void *d_X,
                           pipnn_stream_t stream);

/* (sync) Insert the n_new points the caller has written to rows
 * [n, n + n_new) of X (n = the current point count), which becomes
 * n + n_new. The paper has no insertion; this follows its leaf step:
 *  1. the new rows get norms, sketches, GEMM operand and empty reservoirs;
 *  2. each new point is routed to its fanout[0] nearest leaves of the last
 *     pipnn_build_leaves, by each leaf's representative (the member nearest
 *     to the leaf mean);
 *  3. per (leaf, group) the new points of that group routed to the leaf are
 *     the rows of one rectangular leaf-kernel job whose columns are the
 *     leaf's members and those new points; each row keeps its k nearest
 *     (same GEMM precision, rescoring and selection as the build);
 *  4. both directed records of every pick go through HashPrune;
 *  5. RobustPrune runs again on every point that received a record.
 * d_group (n_new int32, may be NULL = one group) separates requests: new
 * points of different groups are never each other's candidates, so a
 * request gives the same graph whether it is inserted alone or with others
 * (HashPrune does not depend on the order of its records). The leaves
 * themselves do not grow. ESTATE before any build or under capture;
 * EOVERFLOW past the reserved capacity; EINVAL if a leaf would exceed 65535
 * columns. A failed call leaves the point count (and the exactness checks
 * of X) as they were, and the old points' reservoirs and graph rows
 * untouched when it fails before step 4 (every argument and size check
 * does), so the caller may retry with other points in the same rows; the
 * new rows' buffers are rewritten by the next insertion.
 * epoch: the caller's label of the snapshot this insertion publishes; it
 * must exceed the label of the last committed insertion (the index starts
 * at 0), EINVAL otherwise, so that insertions commit in the caller's order.
 * On success (n_new = 0 included) it becomes the index's epoch, reported
 * with the point count by pipnn_get_stats; a failed call keeps the old one. */
pipnn_status pipnn_insert(pipnn_index *idx, int64_t n_new, const int32_t *d_group,
                          uint64_t *d_reservoirs, uint32_t *d_graph, uint32_t *d_degree,
                          uint64_t epoch, pipnn_stream_t stream);

/* Pick + Prune_And_Add_Edges for every leaf (Alg. 4, the parallel loop over
 * leaves; Sec. 4.2): per leaf, the distance matrix on MFMA, each member's
 * k nearest co-members by (GEMM distance, id) (or the rescore_mult*k or
 * k + rescore_extra nearest, rescored), the FP32 direct-difference
 * distance of each winner (for the inner product on an operand equal to the
 * data -- FP32, or fp16 / bf16 data with the same gemm_prec -- the GEMM's
 * own FP32 sum, which has no norm-expansion cancellation to repair; for
 * squared L2 without rescoring on data the integer check found exact -- see
 * pipnn_stats.data_int_exact -- the GEMM distance, which then is the same
 * integer), and both directed records of each picked edge inserted into
 * HashPrune. With leaf_picker ALL_TO_ALL each member
 * instead keeps the candidates that RobustPrune over its whole leaf admits
 * (distances from the leaf's GEMM distance matrix, emitted as FP32 direct
 * differences unless the two forms agree), each giving one record
 * (member, candidate); EINVAL on a leaf of more than 2,048 members.
 * d_leaf_offsets/d_leaf_members is any CSR of leaves with ascending member
 * ids (RBC output or explicit leaves); leaves of size 1 contribute nothing.
 * d_reservoirs holds n x l_max uint64 slots (see pipnn_reservoir_init);
 * repeated calls accumulate, and by the history-independence theorem of
 * Sec. 3 the result does not depend on leaf order or call splitting.
 * Reads d_leaf_offsets back to the host once, unless the same leaves were
 * planned (pipnn_plan_leaves): then it only launches device work and may
 * run under stream capture (it must, if the stream is capturing: ESTATE
 * otherwise). Ties between equal distances go to the co-member at the
 * smaller position in the leaf, which is the smaller id when leaves are
 * ascending. EINVAL on a leaf of more than 65535 points or non-monotone
 * offsets. */
pipnn_status pipnn_build_leaves(pipnn_index *idx, const int64_t *d_leaf_offsets,
                                const uint32_t *d_leaf_members, int64_t n_leaves,
                                uint64_t *d_reservoirs, pipnn_stream_t stream);

/* HashPrune insertion (Alg. 3) of a batch of candidate records
 * (p = d_dst[i], c = d_cand[i], ||p,c|| = d_dist[i]) into the reservoirs.
 * The hash h_p(c) comes from the index's sketches (bit b set iff
 * Sketch(c)_b >= Sketch(p)_b). The stored distance is bf16 (round to nearest
 * even, -0 as +0) and every comparison uses the key (bf16 distance, id).
 * Records with dst == cand are ignored; inserting a record twice changes
 * nothing. Records naming an id >= n are skipped and reported as EDEVICE
 * by this call (it synchronises to read the device-side check); the other
 * records are still inserted. */
pipnn_status pipnn_hashprune_insert(pipnn_index *idx, const uint32_t *d_dst,
                                    const uint32_t *d_cand, const float *d_dist,
                                    int64_t n_records, uint64_t *d_reservoirs,
                                    pipnn_stream_t stream);

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc: tight serving loops, harnesses that forbid allocation): the
 * same insertion as pipnn_hashprune_insert, through the same kernels, with
 * its scratch (per-point counts and bin offsets, the binned records) taken
 * from a fixed array of 64 MiB that the library holds on each device from
 * its load until the process ends. It calls no hipMalloc or hipFree.
 * Limit: the scratch it needs -- 8 (n + 1) bytes of bin offsets,
 * 8 (ceil(n / 4096) + 1) of scan workspace and 4 n of counts, each rounded
 * up to a multiple of 256, plus 8 n_records of binned records -- must not
 * exceed 64 MiB (about 6.8 million records at n = 1,000,000); EINVAL with
 * the sizes otherwise, or if the current device is not the one the index
 * was created on.
 * Every call on a device shares that device's array and leaves its contents
 * behind (each call clears what it needs): calls that overlap in time on one
 * device -- on different streams, threads or indices -- race and must be
 * serialised by the caller. Synchronises the stream like
 * pipnn_hashprune_insert (to read the device-side id check). */
pipnn_status pipnn_hashprune_insert_static(pipnn_index *idx, const uint32_t *d_dst,
                                           const uint32_t *d_cand, const float *d_dist,
                                           int64_t n_records, uint64_t *d_reservoirs,
                                           pipnn_stream_t stream);

/* Reservoir slot layout (Sec. 3, Implementation: 4-byte id, 2-byte hash,
 * bf16 distance): bits 0..31 id, 32..47 hash, 48..63 bf16 distance.
 * Sets n x l_max slots to the empty slot (id 0xFFFFFFFF, hash 0, +inf). */
pipnn_status pipnn_reservoir_init(uint64_t *d_reservoirs, int64_t n, int32_t l_max,
                                  pipnn_stream_t stream);

/* Writes the canonical form of the reservoirs: per point, valid slots
 * sorted by (bf16 distance, id) and empty slots last. Reservoirs written by
 * this library are already canonical; d_out may equal d_res. */
pipnn_status pipnn_reservoir_canonical(const pipnn_index *idx, const uint64_t *d_res,
                                       uint64_t *d_out, pipnn_stream_t stream);

/* Final prune (Alg. 4, PruneNode; Sec. 4.3): RobustPrune (Alg. 2) in its
 * lazy form (Supplement, "Optimizing RobustPrune") on every reservoir. The
 * candidates of x are its reservoir ids; d(x,c) is the FP32 direct-
 * difference distance, and d(y,c) between candidates the FP32 GEMM form
 * |y|^2 + |c|^2 - 2 y.c (or -y.c) from a Gram on MFMA (up to 64 candidates
 * and 128 dimensions; the 16-bit copy of X when it holds X exactly, see
 * gemm_prec), for 512 / 768-dimension bf16 / fp16 operands both come from
 * the operand's Gram, and otherwise both are direct differences. With the
 * int8 rows (L2, integral X spanning at most 256 values, d <= 128,
 * l_max <= 64, alpha < 2^23) every distance is an exact integer (dot4
 * products and an int8 Gram on MFMA), and the test alpha*d(y,c) < d(x,c)
 * is taken exactly in integers; pipnn_stats.rp_row_bits names the row
 * width read (8, 16 or 32).
 * Candidates are taken in (d(x,c), id) order and c is admitted unless an
 * admitted y has alpha*d(y,c) < d(x,c) (evaluated as the sign of one fused
 * multiply-add, or exactly in integers on the int8 rows). Writes d_graph
 * (n x R, admission order, 0xFFFFFFFF padding) and d_degree (n). */
pipnn_status pipnn_robustprune(pipnn_index *idx, const uint64_t *d_reservoirs, uint32_t *d_graph,
                               uint32_t *d_degree, pipnn_stream_t stream);

/* (sync) The search start point: the point nearest the mean of X by
 * (squared L2, id), the mean and distances in FP64. Written to *h_out. */
pipnn_status pipnn_start_node(pipnn_index *idx, uint32_t *h_out, pipnn_stream_t stream);

/* BeamSearch (Alg. 1) for nq queries d_Q (nq x d, q_dtype) over d_graph
 * (n x R from pipnn_robustprune) from start point `start`, beam width L.
 * Writes the first k beam entries per query: d_out_ids (nq x k) and
 * d_out_dist (nq x k, FP32; may be NULL); d_out_cmps (nq, may be NULL)
 * receives the number of distance evaluations, the start included.
 * EINVAL if k < 1, k > L, L > 1024, start >= n. */
pipnn_status pipnn_search(pipnn_index *idx, const uint32_t *d_graph, const void *d_Q, int64_t nq,
                          int32_t q_dtype, int32_t k, int32_t L, uint32_t start,
                          uint32_t *d_out_ids, float *d_out_dist, uint32_t *d_out_cmps,
                          pipnn_stream_t stream);

/* Approximate k-nearest-neighbour graph of the indexed points (Sec. 5, k-NN
 * graph construction: build the index, then search every point): for each
 * point p, BeamSearch (Alg. 1, as pipnn_search) for X[p] with beam width L
 * from `start` returns its k + 1 nearest, and p itself is dropped (or, when
 * p is not among them, the (k + 1)-th). Writes d_out_ids (n x k, ids in
 * (distance, id) order) and d_out_dist (n x k FP32 distances; may be NULL).
 * Points are searched in chunks of up to 65,536. EINVAL unless
 * 1 <= k < L <= 1024 and start < n. */
pipnn_status pipnn_knn_graph(pipnn_index *idx, const uint32_t *d_graph, int32_t k, int32_t L,
                             uint32_t start, uint32_t *d_out_ids, float *d_out_dist,
                             pipnn_stream_t stream);

/* Recompute the per-point squared norms and sketches from X (call after the
 * caller changed X in place; pipnn_create already does this once), with the
 * integer check of X (every coordinate an integer, d*A^2 <= 2^23 and
 * d*W^2 <= 2^24 for the largest magnitude A and the range W; read back
 * with one synchronization, except under stream capture, where the last
 * result is kept). */
pipnn_status pipnn_prepare(pipnn_index *idx, pipnn_stream_t stream);

/* Counters and phase timings of the most recent calls on an index.
 * Phase times (milliseconds, summed since profiling was switched on) are
 * taken with HIP events recorded on the call's stream around each phase:
 * ms_leaf_knn covers only the fused leaf distance + selection kernel. */
typedef struct {
  int64_t n_leaves, n_members;   /* last pipnn_partition */
  int64_t leader_dists;          /* point-to-leader distances it evaluated */
  int32_t levels;                /* its recursion levels */
  int32_t leaf_knn_launches;     /* leaf kernel launches since profiling on */
  int64_t leaf_pairs;            /* sum of s^2 over the leaves of the last build */
  int64_t records;               /* candidate records binned by the last build */
  int32_t operand_exact;         /* 1: the 16-bit or reduced-precision copy of X (the GEMM
                                    operand, or a float32 index's fp16 copy) holds X exactly
                                    and is used where the gemm_prec notes say */
  int32_t data_int_exact;        /* 1: X is integral with a range that makes every squared-L2
                                    form exact in float32, so the leaf picks skip the winners'
                                    FP32 recompute (no rescoring) */
  double ms_prepare, ms_partition, ms_leaf_knn, ms_bin, ms_merge, ms_robustprune;
  uint64_t epoch;                /* epoch of the last committed pipnn_insert (0: none) */
  int64_t n_points;              /* current point count */
  int64_t workspace_bytes;       /* the workspace layout in use (0: the index allocates) */
  int64_t batch_rows;            /* leaf rows per pick + binning batch of a build */
  int32_t rp_row_bits;           /* element width of the rows pipnn_robustprune reads: 8 (the
                                    int8 rows of an integral float32 X spanning <= 256 values,
                                    L2), 16 (the exact 16-bit copy) or 32 (float32) */
  int32_t reserved_;
} pipnn_stats;

/* Switch phase timing on (1; also clears the sums) or off (0). */
pipnn_status pipnn_set_profiling(pipnn_index *idx, int32_t on);

/* (sync) Fills *h_out; synchronises the recorded events. */
pipnn_status pipnn_get_stats(pipnn_index *idx, pipnn_stats *h_out);

/* ---- inspection calls, used to check the path against the oracle ---- */

/* Copies the index's float32 sketches (n x hash_bits) to d_out. */
pipnn_status pipnn_get_sketches(const pipnn_index *idx, float *d_out, pipnn_stream_t stream);

/* The leaf distance kernel on one explicit block: rows d_row_ids (n_rows
 * point ids) against columns d_col_ids (n_cols point ids), each row's
 * k nearest columns by (GEMM distance, column index), excluding the column
 * at the row's own position when exclude_diag is 1 (then n_rows must equal
 * n_cols and the two lists must be equal). Writes column indices
 * d_out_col (n_rows x k) in that order, the FP32 direct-difference
 * distances d_out_dist (n_rows x k, may be NULL) and, when d_out_matrix is
 * not NULL, the GEMM distances of every pair (n_rows x n_cols). The same
 * code as pipnn_build_leaves runs, with the index's gemm_prec and
 * rescoring. EINVAL if k < 1, the selected count (k, rescore_mult * k or
 * k + rescore_extra) > 32, n_cols > 65535. */
pipnn_status pipnn_knn_block(pipnn_index *idx, const uint32_t *d_row_ids, int64_t n_rows,
                             const uint32_t *d_col_ids, int64_t n_cols, int32_t k,
                             int32_t exclude_diag, uint32_t *d_out_col, float *d_out_dist,
                             float *d_out_matrix, pipnn_stream_t stream);

/* The pick step alone: like pipnn_build_leaves but, instead of inserting
 * into HashPrune, writes each leaf row's picks as point ids d_out_cand and
 * FP32 direct-difference distances d_out_dist, both (offsets[L] x k) in CSR
 * member order, unused slots 0xFFFFFFFF / +inf. With leaf_picker ALL_TO_ALL
 * the picks are the admitted candidates in admission order. */
pipnn_status pipnn_leaf_pick(pipnn_index *idx, const int64_t *d_leaf_offsets,
                             const uint32_t *d_leaf_members, int64_t n_leaves, uint32_t *d_out_cand,
                             float *d_out_dist, pipnn_stream_t stream);

/* The reduced-precision leaf-GEMM operand the index made from X (gemm_prec
 * BF16, FP16 or FP8): d_codes (n x d; uint16 bf16 / fp16 bits, or uint8
 * OCP e4m3 codes), d_scale (n floats: the per-point decode scale, value =
 * code * scale, max|x_i| / 448 for fp8 and 1 otherwise) and d_norms (n
 * floats: squared norms of the decoded vectors, the norms the GEMM form
 * uses). Any output may be NULL. ESTATE if gemm_prec is FP32. */
pipnn_status pipnn_get_operand(const pipnn_index *idx, void *d_codes, float *d_scale,
                               float *d_norms, pipnn_stream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* PIPNN_H */

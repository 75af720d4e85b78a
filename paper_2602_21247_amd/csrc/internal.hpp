// Host-side structures of the PiPNN gfx950 library and the launchers each
// kernel file provides.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <deque>
#include <string>
#include <vector>

#include "../../include/pipnn.h"

namespace pipnn {

// A device buffer owned by the index; grows on demand, never shrinks.
// On an index created over a caller's workspace the buffer is `fixed`: its
// slice of the workspace (ws_p, lim bytes) is set at creation, ensure()
// hands it out on first use and fails with hipErrorOutOfMemory for a
// request above lim; nothing is ever allocated.
struct DevBuf {
  void *p = nullptr;
  size_t cap = 0;
  void *ws_p = nullptr;  // the fixed slice (fixed buffers)
  size_t lim = 0;        // its size in bytes
  bool fixed = false;
  hipError_t ensure(size_t bytes);
  void release();
  template <class T> T *as() const { return reinterpret_cast<T *>(p); }
};

// Pinned host staging for the small tables a call uploads (work lists,
// segment tables): each table is appended to one pinned buffer and copied
// to its device buffer asynchronously, so the host need not wait for the
// copy; the buffer is reused from the start only after the stream has been
// synchronised (reset), and a table that does not fit synchronises first.
// Host memory only (an index on a workspace allocates no device memory).
struct HostStage {
  uint8_t *p = nullptr;
  size_t cap = 0, used = 0;
  hipError_t put(DevBuf &dst, const void *src, size_t bytes, hipStream_t s);
  void reset() { used = 0; }
  void release();
};

struct Index {
  pipnn_params p;
  HostStage stage;           // pinned staging of uploaded tables
  bool ws_mode = false;      // every DevBuf is a fixed slice of the caller's workspace
  size_t ws_bytes = 0;       // the layout's total (ws_mode)
  int64_t batch_rows = (int64_t)1 << 25;  // leaf rows per pick + binning batch
  uint64_t epoch = 0;        // the caller's label of the last committed insertion
  const void *X = nullptr;  // n x d, caller-owned
  int64_t n = 0;
  int32_t d = 0;
  int32_t x_dtype = PIPNN_DTYPE_F32;
  const float *H = nullptr;  // m x d, caller-owned
  int32_t m = 0;
  hipStream_t stream = nullptr;

  DevBuf xf32;      // float32 copy of X when X is not float32
  DevBuf xlow;      // low-precision copy of X (copy_prec): the leaf GEMM operand of a reduced
                    // gemm_prec; for a float32 index of at most 128 dimensions an fp16 copy
                    // kept while X is integral (int_exact), used where it holds X exactly
  int32_t copy_prec = PIPNN_PREC_FP32;  // the format of xlow (FP32: none)
  DevBuf xscale;    // per-point fp8 decode scale (value = code * scale)
  DevBuf lnorms;    // n float32, squared norms of the decoded low-precision operand
  DevBuf op_flag;   // int32: set by the encoder when a value does not survive encoding
  bool op_exact = false;  // the reduced-precision operand holds X exactly
  // Integer check of X, taken with the norms: int32 [not integral or
  // |v| > 2^20, min, max]; int_exact when every coordinate is an integer
  // and the range keeps every distance form exact in float32.
  DevBuf int_chk;
  bool int_exact = false;
  int64_t int_lo = 0, int_hi = 0;
  int32_t ldo = 0;  // row stride (elements) of xlow: d padded by lowp_padded_dim
  // int8 rows for RobustPrune (L2, float32 index of at most 128 dimensions):
  // while X is integral and every coordinate lies in [lo8, lo8 + 255], row
  // p holds x_p - lo8 - 128 (zero padded to ld8 bytes) and n8 its squared
  // norm; distances are translation invariant, so every L2 distance form
  // is the same integer on these rows
  DevBuf x8, n8;
  int32_t ld8 = 0;
  int64_t lo8 = 0;
  bool i8_ok = false;
  DevBuf xpad;      // float32 GEMM operand zero padded to ldf, when X itself cannot serve
  int32_t ldf = 0;  // row stride (floats) of the float32 GEMM operand; 0: d > 256
  DevBuf sketches;  // n x m float32
  DevBuf norms;     // n float32, squared norms of the float32 vectors
  DevBuf flag;      // int32 device error flag

  // scratch reused across calls
  DevBuf s_jobs, s_items, s_picks_c, s_picks_d, s_cnt, s_off, s_bins, s_tmp0, s_tmp1;
  // partition (one level at a time): the members of the level's
  // subproblems (ping-pong), their leader assignments, the assignments
  // grouped by bucket, the merged small buckets and their sizes, and the
  // host-built tables of the merge, recursion and leaf-output copies
  DevBuf p_mem[2], p_asg, p_G, p_gout, p_gsize;
  DevBuf p_leaders, p_cm, p_bstart, p_groups;
  DevBuf p_seg, p_seglen, p_segfirst, p_segoff, p_rsrc, p_roff, p_rlen, p_esrc, p_eoff, p_elen;
  DevBuf rp_order;              // RobustPrune processing order (from the last leaves)
  DevBuf s_counter;             // per-XCD work counters of the persistent leaf schedule
  // the leaves of the last build, kept for insertion: CSR rebased to 0 (a
  // host copy of the offsets too) and one representative member per leaf
  DevBuf lt_off, lt_mem, lt_rep;
  std::vector<int64_t> lt_offs;
  int64_t lt_n_leaves = 0;
  bool lt_reps_valid = false;
  int64_t cap = 0;              // rows the per-point buffers hold (pipnn_reserve)
  DevBuf i_rows, i_cols, i_assign, i_flag, i_pos, i_list, i_tmp, i_segs;
  DevBuf q_conv, q_seen;        // search scratch (search may overlap an insertion)
  DevBuf g_ids, g_dist;         // k-NN graph: k + 1 results per point of a chunk
  DevBuf a2a_mat, a2a_tmp;      // all-to-all picker: leaf distance matrices of a batch
  int32_t device = 0;           // the HIP device current at pipnn_create
  int32_t n_cu = 256;           // compute units of the device (persistent grid size)
  int32_t leaf_nw = 4;          // waves (of 32 rows) per leaf work item: 4, or 2 where built
  int32_t leaf_persistent = 0;  // 1: persistent workgroups take items from the counters
  int32_t leaf_quad = 0;        // 1: four lanes per row (128-row items)
  // A planned leaf set (pipnn_plan_leaves): its work lists live on the
  // device, so that pipnn_build_leaves on it does no host work and can be
  // captured in a graph.
  struct PlanBatch {
    int64_t l0 = 0, l1 = 0, rows = 0, pairs = 0;
    int64_t job_off = 0, item_off = 0;  // the batch's work lists in jobs / items
    int32_t n_items = 0, max_cols = 0;
  };
  struct LeafPlan {
    const int64_t *d_off = nullptr;
    const uint32_t *d_mem = nullptr;
    int64_t n_leaves = -1;
    int32_t nw = 0;
    std::vector<int64_t> offs;
    std::vector<PlanBatch> batches;
    DevBuf jobs, items;  // every batch's work lists, one after another
  } plan;
  DevBuf o_first, o_flag, o_pos, o_pos2, o_tmp;
  bool rp_order_valid = false;

  // statistics and phase events
  pipnn_stats stats{};
  bool profiling = false;
  struct Ev {
    int phase;
    hipEvent_t a, b;
  };
  std::vector<Ev> events;
  std::vector<hipEvent_t> ev_free;
  double phase_ms[8] = {0};
  int leaf_launches = 0;

  // The exact 16-bit copy serves the partition's leader distances and
  // RobustPrune's rows: for a bf16 / fp16 index when it holds X exactly; for
  // a float32 index when it holds X exactly and X passed the integer check
  // (then every distance form is the same integer in either format).
  bool copy16_exact() const {
    if (!xlow.p || !op_exact) return false;
    if (copy_prec != PIPNN_PREC_BF16 && copy_prec != PIPNN_PREC_FP16) return false;
    return p.gemm_prec != PIPNN_PREC_FP32 || int_exact;
  }
  const float *xf() const;
  const float *xop32() const;  // the float32 GEMM operand: xpad if allocated, else xf()
};

// Phase timing: begin/end record events on the stream when profiling is on.
enum Phase { kPhPrepare = 0, kPhPartition, kPhLeafKnn, kPhBin, kPhMerge, kPhRobustPrune };
bool stream_capturing(hipStream_t s);
struct PhaseTimer {
  Index &I;
  int phase;
  hipStream_t s;
  hipEvent_t a = nullptr;
  PhaseTimer(Index &I_, int ph, hipStream_t s_);
  ~PhaseTimer();
};

// ---- knn (fused distance GEMM + per-row selection) --------------------
struct KnnJob {
  int64_t row_off;   // into row_base
  int64_t col_off;   // into col_base
  int64_t out_off;   // first output row
  int32_t n_rows, n_cols;
  int32_t k_sel;     // number of GEMM-nearest kept (<= KSEL)
  int32_t flags;     // bit 0: exclude column self_off + r for row r (the row itself)
  int32_t self_off;  // column of row 0 when bit 0 is set
  int32_t pad_;
};
struct KnnItem {
  int32_t job, rb;
};

struct KnnLaunch {
  const Index *idx;
  const uint32_t *row_base, *col_base;
  const KnnJob *jobs;
  const KnnItem *items;
  int32_t n_items;
  int32_t max_cols;      // largest n_cols over the jobs
  int32_t ksel;          // selection size used to pick the template
  int32_t k_out;         // outputs per row
  int32_t out_ids;       // 1: write col_base ids, 0: write column indices
  int32_t recompute;     // 1: FP32 direct-difference distance of the winners
  int32_t rescore_k;     // > 0: keep this many of the k_sel by the direct distance
  int32_t prec;          // PIPNN_PREC_*: the operand (FP32 for the partition)
  int32_t nw;            // waves per work item (rows per item / 32)
  int32_t persistent;    // 1: persistent schedule over Index::s_counter
  int32_t quad = 0;      // 1: four lanes per row (knn_quad.hpp), on 128-row items
  uint32_t *out_col;
  float *out_dist;
  float *out_matrix;
  int64_t matrix_ld;
};
hipError_t launch_knn(const KnnLaunch &L, hipStream_t s);
// Operand width the leaf kernel is instantiated for (0: not supported), and
// whether work items of 32 * nw rows exist for it.
int knn_operand_dim(int d, int prec);
bool knn_nw_available(int d, int prec, int nw);
// Whether the four-lane layout is built for the operand, and the two-lane one.
bool knn_quad_available(int d, int prec);
bool knn_pair_available(int d, int prec);

// Reduced-precision operands are stored zero padded to one of these
// dimensions, so that every operand row is a whole number of 16-byte
// vectors and the kernel never tests the dimension; 0 = not supported.
inline int lowp_padded_dim(int d) {
  return d <= 64 ? 64 : d <= 96 ? 96 : d <= 128 ? 128 : d <= 256 ? 256 : d <= 512 ? 512
       : d <= 768 ? 768 : 0;
}

// Bytes per int8 row (d <= 128): 64 or 128, so that a row is whole MFMA
// k-steps of 32 split over the two half-waves.
inline int rows8_width(int d) { return d <= 64 ? 64 : 128; }

// ---- misc kernels ----------------------------------------------------
hipError_t launch_norms_sketches(const Index &I, hipStream_t s);
// The index's reduced-precision operand (I.p.gemm_prec): codes into I.xlow
// (n x I.ldo), decode scales into I.xscale (fp8), squared norms of the
// decoded vectors into I.lnorms.
hipError_t launch_quantize(const Index &I, hipStream_t s);
// the same for points [p0, p0 + cnt) only
hipError_t launch_norms_sketches_range(const Index &I, int64_t p0, int64_t cnt, hipStream_t s);
hipError_t launch_quantize_range(const Index &I, int64_t p0, int64_t cnt, hipStream_t s,
                                 bool with8 = false);
// The int8 rows and their norms (I.x8, I.n8) of points [p0, p0 + cnt)
// (launch_quantize_range with with8 writes them in its own pass where it can).
hipError_t launch_quantize8_range(const Index &I, int64_t p0, int64_t cnt, hipStream_t s);
// Clear the encoder's inexact flag (a fill kernel, so it may be captured),
// and, outside capture, read it back into I.op_exact (synchronizes s):
// `reset` clears op_exact first for a full re-encode.
hipError_t clear_op_flag(Index &I, hipStream_t s);
hipError_t clear_int_check(Index &I, hipStream_t s);
// (sync) reads the integer check of the points normed since the last clear;
// reset: those are all the points, else they are added to the earlier ones
hipError_t read_int_check(Index &I, bool reset, hipStream_t s);
hipError_t read_op_flag(Index &I, bool reset, hipStream_t s);
// Rows [p0, p0 + cnt) of the zero-padded float32 operand I.xpad.
hipError_t launch_pad_range(const Index &I, int64_t p0, int64_t cnt, hipStream_t s);
// leaf table: offsets rebased to 0, member copy, one representative per leaf
hipError_t launch_rebase_i64(const int64_t *in, int64_t n, int64_t *out, hipStream_t s);
hipError_t launch_copy_u32(const uint32_t *in, int64_t n, uint32_t *out, hipStream_t s);
hipError_t launch_leaf_reps(const float *X, int d, const int64_t *off, const uint32_t *mem,
                            int64_t n_leaves, uint32_t *rep, hipStream_t s);
// flag[v] = 1 for every id v < n in ids; out[pos[i]] = i for flagged i
hipError_t launch_mark_ids(const uint32_t *ids, int64_t cnt, int64_t n, uint32_t *flag,
                           hipStream_t s);
hipError_t launch_compact_flags(const uint32_t *flag, const int64_t *pos, int64_t n, uint32_t *out,
                                hipStream_t s);
hipError_t launch_to_f32(const void *src, int dtype, float *dst, int64_t count, hipStream_t s);
hipError_t launch_iota(uint32_t *dst, int64_t n, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *dst, uint32_t v, int64_t n, hipStream_t s);
hipError_t launch_fill_u64(uint64_t *dst, uint64_t v, int64_t n, hipStream_t s);
// exclusive scan of n uint32 into n+1 int64 (out[n] = total); tmp holds
// scan_tmp_elems(n) int64
int64_t scan_tmp_elems(int64_t n);
hipError_t launch_scan_u32(const uint32_t *in, int64_t *out, int64_t n, int64_t *tmp, hipStream_t s);
hipError_t launch_scan_i64_inplace(int64_t *data, int64_t n, int64_t *tmp, hipStream_t s);
hipError_t launch_gather_u32(const uint32_t *src, const int64_t *idx, uint32_t *dst, int64_t n,
                             hipStream_t s);

// ---- partition group-by ------------------------------------------------
struct GroupSub {
  int64_t elem_off;   // first element (instance x fanout slot) of the subproblem
  int64_t n_elems;
  int64_t cm_off;     // first counter of its (bucket x tile) matrix
  int32_t n_buckets;  // leaders
  int32_t n_tiles;
  int64_t bucket_off; // first global bucket index
};
struct GroupTile {
  int32_t sub, tile;
};
hipError_t launch_groupby(const uint32_t *asg_col, const uint32_t *src_ids, int32_t *fan,
                          const GroupSub *subs, const GroupTile *tiles, int32_t n_tiles,
                          int32_t tile_elems, int64_t *cm, int64_t cm_len, int64_t *tmp,
                          uint32_t *out, int64_t *bucket_start, int64_t n_buckets_total,
                          int32_t max_buckets, hipStream_t s);
struct MergeGroup {
  int64_t src_off[1];
};
hipError_t launch_merge_dedup(const uint32_t *const *seg_ptr, const int32_t *seg_len,
                              const int32_t *grp_first_seg, int32_t n_groups, int32_t max_sum,
                              uint32_t *out, const int64_t *out_off, int32_t *out_size,
                              hipStream_t s);
hipError_t launch_copy_segments(const uint32_t *const *src, const int64_t *dst_off,
                                const int32_t *len, int32_t n_segs, uint32_t *dst, hipStream_t s);

// ---- HashPrune -------------------------------------------------------
// Leaf-local binning of the picks of leaves [0, n_leaves) of a batch
// (leaf_off: their absolute offsets, off0 the batch's first row; picks as
// local column indices): count pass (scatter = false: adds to cnt) or
// scatter pass (cnt as the per-point cursor, bins at bin_off).
constexpr int kLeafBinMaxRows = 4096;
hipError_t launch_leaf_bin(bool scatter, const int64_t *leaf_off, int64_t off0, int64_t n_leaves,
                           const uint32_t *members, const uint32_t *picks, const float *dist,
                           int32_t k, const float *sketch, int32_t m, const int64_t *bin_off,
                           uint32_t *cnt, uint64_t *bins, hipStream_t s);
// bidir: every pick (i -> j) yields the records (i, j) and (j, i); else
// only (i, j)
hipError_t launch_bin_count(const uint32_t *row_ids, const uint32_t *picks, int64_t n_rows,
                            int32_t k, uint32_t *cnt, int64_t n, int32_t *flag, hipStream_t s,
                            bool bidir = true);
hipError_t launch_bin_scatter(const uint32_t *row_ids, const uint32_t *picks, const float *dist,
                              int64_t n_rows, int32_t k, const float *sketch, int32_t m,
                              const int64_t *off, uint32_t *cursor, uint64_t *bins, int64_t n,
                              hipStream_t s, bool bidir = true);
hipError_t launch_rec_count(const uint32_t *dst, const uint32_t *cand, int64_t cnt_rec,
                            uint32_t *cnt, int64_t n, int32_t *flag, hipStream_t s);
hipError_t launch_rec_scatter(const uint32_t *dst, const uint32_t *cand, const float *dist,
                              int64_t cnt_rec, const float *sketch, int32_t m, const int64_t *off,
                              uint32_t *cursor, uint64_t *bins, int64_t n, hipStream_t s);
hipError_t launch_hashprune_merge(uint64_t *res, int64_t n, int32_t l_max, const uint64_t *bins,
                                  const int64_t *off, hipStream_t s);
hipError_t launch_reservoir_canonical(const uint64_t *in, uint64_t *out, int64_t n, int32_t l_max,
                                      hipStream_t s);

// ---- RobustPrune / search ---------------------------------------------
// RobustPrune of every point (subset NULL; in leaf order when known) or of
// the n_subset points listed in subset.
// Element width (8, 16 or 32 bits) of the rows launch_robustprune reads.
int rp_row_bits(const Index &I);
hipError_t launch_robustprune(const Index &I, const uint64_t *res, uint32_t *graph, uint32_t *degree,
                              const uint32_t *subset, int64_t n_subset, hipStream_t s);
hipError_t launch_leaf_order(const uint32_t *mem, int64_t cnt, int64_t n, uint32_t *first,
                             uint32_t *flag, int64_t *pos, int64_t *pos2, int64_t *tmp,
                             uint32_t *order, hipStream_t s);
hipError_t launch_start_node(const Index &I, double *tmp, uint32_t *out, hipStream_t s);
// n: the point count the graph covers (ids >= n are not visited)
hipError_t launch_search(const Index &I, int64_t n, const uint32_t *graph, const float *Q,
                         int64_t nq, int32_t k, int32_t L, uint32_t start, uint32_t *out_ids,
                         float *out_dist, uint32_t *out_cmps, uint32_t *visited_bits,
                         int64_t words_per_query, hipStream_t s);

// All-to-All Prune picks of the rows [off0, off0 + rows) of a batch of
// leaves (leaf_off: absolute offsets of the batch's n_leaves leaves) from
// their GEMM distance matrices D (row r at D + r * ld, column = position in
// the leaf): out_id / out_dist rows x R (point ids in admission order).
hipError_t launch_a2a_prune(const float *D, int64_t ld, const int64_t *leaf_off, int64_t n_leaves,
                            int64_t off0, int64_t rows, const uint32_t *members, const float *X,
                            int32_t d, int32_t metric, int32_t recompute, int32_t R, float alpha,
                            uint32_t *out_id, float *out_dist, hipStream_t s);
constexpr int kA2aMaxLeaf = 2048;

// k + 1 results per point searched as a query -> k without the point itself
hipError_t launch_drop_self(const uint32_t *ids, const float *dist, int64_t nq, int32_t k1,
                            int64_t q0, uint32_t *out_ids, float *out_dist, hipStream_t s);

}  // namespace pipnn

// C ABI of the PiPNN gfx950 library and its host-side orchestration.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <deque>
#include <new>
#include <string>
#include <vector>

#include "common.hpp"
#include <map>
#include <mutex>

#include "internal.hpp"

using namespace pipnn;

namespace {

thread_local std::string g_err;

pipnn_status fail(pipnn_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIPCHK(expr)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return fail(e_ == hipErrorOutOfMemory ? PIPNN_ENOMEM : PIPNN_EDEVICE, "%s failed: %s", \
                  #expr, hipGetErrorString(e_));                                              \
  } while (0)

}  // namespace

namespace pipnn {
bool stream_capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(s, &st) == hipSuccess && st == hipStreamCaptureStatusActive;
}
}  // namespace pipnn

namespace {

#define GUARD_BEGIN try {
#define GUARD_END                                                    \
  }                                                                  \
  catch (const std::bad_alloc &) {                                   \
    return fail(PIPNN_ENOMEM, "host allocation failed");             \
  }                                                                  \
  catch (...) {                                                      \
    return fail(PIPNN_EDEVICE, "unexpected internal exception");    \
  }

// splitmix64 (Steele, Lea and Flood, 2014): golden-ratio increment of the
// state, then the published xor-shift-multiply finaliser.
uint64_t sm64_next(uint64_t &state) {
  uint64_t z = (state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Root key of partition replica r: the seed itself for r = 0, else the
// first splitmix64 output from the seed xor r times a second odd constant
// (distinct from the child-key constant below).
uint64_t replica_key(uint64_t seed, int64_t r) {
  if (r == 0) return seed;
  uint64_t s = seed ^ ((uint64_t)r * 0xD1B54A32D192ED03ull);
  return sm64_next(s);
}

// Key of the subproblem formed by bucket t of a subproblem with key `key`.
uint64_t sub_key(uint64_t key, int64_t t) {
  uint64_t s = key ^ ((uint64_t)(t + 1) * 0x9E3779B97F4A7C15ull);
  return sm64_next(s);
}

// Positions (within the subproblem's ascending id list) of its `ell`
// leaders: the first ell entries of a partial Fisher-Yates shuffle driven by
// splitmix64 from `key`, drawing j = t + floor(r * (np - t) / 2^64) (Alg. 5,
// SampleLeaders). Only swapped positions are stored, in an open-addressing
// table (linear probing, at most half full).
std::vector<int64_t> leader_positions(uint64_t key, int64_t np, int64_t ell) {
  size_t cap = 16;
  while (cap < (size_t)ell * 4) cap <<= 1;
  const size_t mask = cap - 1;
  std::vector<int64_t> keys(cap, -1), vals(cap);
  auto slot = [&](int64_t i) {
    size_t h = (size_t)(((uint64_t)i * 0x9E3779B97F4A7C15ull) >> 20) & mask;
    while (keys[h] != -1 && keys[h] != i) h = (h + 1) & mask;
    return h;
  };
  auto at = [&](int64_t i) {
    const size_t h = slot(i);
    return keys[h] == -1 ? i : vals[h];
  };
  auto put = [&](int64_t i, int64_t v) {
    const size_t h = slot(i);
    keys[h] = i;
    vals[h] = v;
  };
  std::vector<int64_t> pos((size_t)ell);
  uint64_t st = key;
  for (int64_t t = 0; t < ell; ++t) {
    const uint64_t r = sm64_next(st);
    const int64_t j =
        t + (int64_t)(((unsigned __int128)r * (unsigned __int128)(uint64_t)(np - t)) >> 64);
    const int64_t vt = at(t), vj = at(j);
    put(t, vj);
    put(j, vt);
    pos[(size_t)t] = vj;
  }
  return pos;
}

// Whether the leaf pick re-ranks its GEMM winners by the FP32 direct
// difference, and how many it selects by the GEMM distance for k kept:
// rescore_mult * k, or k + rescore_extra (k itself without rescoring).
static bool rescoring(const pipnn_params &P) { return P.rescore_mult != 0 || P.rescore_extra != 0; }
static int sel_count(const pipnn_params &P, int k) {
  return P.rescore_mult ? P.rescore_mult * k : k + P.rescore_extra;
}

bool valid_params(const pipnn_params *p, std::string &why) {
  char b[160];
  auto bad = [&](const char *m) {
    why = m;
    return false;
  };
  if (!p) return bad("params is NULL");
  if (p->metric != PIPNN_METRIC_L2 && p->metric != PIPNN_METRIC_IP) return bad("unknown metric");
  if (p->c_max < 2 || p->c_max > 16384) return bad("c_max must be in 2..16384");
  if (p->c_min < 0 || p->c_min > p->c_max) return bad("c_min must be in 0..c_max");
  if (p->leader_div < 1) return bad("leader_div must be >= 1");
  if (p->leader_cap < 2 || p->leader_cap > 4096) return bad("leader_cap must be in 2..4096");
  for (int i = 0; i < 4; ++i)
    if (p->fanout[i] < 1 || p->fanout[i] > 4) return bad("fanout values must be in 1..4");
  if (p->fanout[3] != 1) return bad("fanout[3] must be 1");
  if (p->k < 1 || p->k > 32) return bad("k must be in 1..32");
  if (p->hash_bits < 1 || p->hash_bits > 16) return bad("hash_bits must be in 1..16");
  if (p->l_max < 1 || p->l_max > 256) return bad("l_max must be in 1..256");
  if (p->R < 1 || p->R > 256) return bad("R must be in 1..256");
  if (!(p->alpha >= 1.0f)) return bad("alpha must be >= 1");
  if (p->gemm_prec != PIPNN_PREC_FP32 && p->gemm_prec != PIPNN_PREC_BF16 &&
      p->gemm_prec != PIPNN_PREC_FP8 && p->gemm_prec != PIPNN_PREC_FP16) {
    snprintf(b, sizeof(b), "unknown gemm_prec %d", p->gemm_prec);
    why = b;
    return false;
  }
  if (p->rescore_mult != 0 && (p->rescore_mult < 2 || p->rescore_mult * p->k > 32))
    return bad("rescore_mult must be 0, or >= 2 with rescore_mult * k <= 32");
  if (p->rescore_extra < 0 || p->k + p->rescore_extra > 32)
    return bad("rescore_extra must be >= 0 with k + rescore_extra <= 32");
  if (p->rescore_mult != 0 && p->rescore_extra != 0)
    return bad("rescore_mult and rescore_extra are alternatives: set at most one");
  if (p->leaf_picker != PIPNN_PICKER_KNN && p->leaf_picker != PIPNN_PICKER_ALL_TO_ALL)
    return bad("unknown leaf_picker");
  if (p->leaf_picker == PIPNN_PICKER_ALL_TO_ALL && rescoring(*p))
    return bad("the all-to-all leaf picker takes no rescoring (rescore_mult and rescore_extra 0)");
  return true;
}

// The same through the index's pinned staging (asynchronous; see HostStage).
template <class T>
hipError_t staged(Index &I, DevBuf &b, const std::vector<T> &v, hipStream_t s) {
  return I.stage.put(b, v.data(), v.size() * sizeof(T), s);
}

template <class T>
hipError_t upload(DevBuf &b, const std::vector<T> &v, hipStream_t s) {
  hipError_t e = b.ensure(std::max<size_t>(1, v.size()) * sizeof(T));
  if (e != hipSuccess || v.empty()) return e;
  return hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
}

constexpr int kGroupTile = 1024;

// Indices 0..n-1 by falling w, equal values by rising index: a stable LSD
// radix sort (8-bit digits) of max(w) - w.
std::vector<int> order_by_falling(const std::vector<uint64_t> &w) {
  const size_t n = w.size();
  uint64_t mx = 0;
  for (uint64_t v : w) mx = std::max(mx, v);
  std::vector<int> a(n), b(n);
  for (size_t i = 0; i < n; ++i) a[i] = (int)i;
  for (int shift = 0; shift < 64 && (mx >> shift) != 0; shift += 8) {
    size_t cnt[257] = {0};
    for (size_t i = 0; i < n; ++i) ++cnt[(((mx - w[(size_t)a[i]]) >> shift) & 255u) + 1];
    for (int k = 0; k < 256; ++k) cnt[k + 1] += cnt[k];
    for (size_t i = 0; i < n; ++i) b[cnt[((mx - w[(size_t)a[i]]) >> shift) & 255u]++] = a[i];
    a.swap(b);
  }
  return a;
}

// Work items of a knn launch in launch order: block b runs on XCD b % 8 and
// takes item b. Jobs are taken largest first (by rows x columns); a job of
// at most 16 row blocks goes whole to the least-loaded XCD (its columns stay
// in that XCD's L2), the row blocks of a larger job are dealt in turn to the
// XCDs in rising order of load. Shorter XCD lists are padded with idle
// items. The first pass fixes each job's XCDs and the list lengths, the
// second writes the items in place. (Every row's result is the same for
// any order of the items: the plan decides only the balance.)
std::vector<KnnItem> plan_items(const std::vector<KnnJob> &jobs, int rows_per_item = 128) {
  constexpr int X = kNumXcd;
  const int64_t rpi = rows_per_item;
  const size_t nj = jobs.size();
  std::vector<uint64_t> work(nj);
  for (size_t i = 0; i < nj; ++i) work[i] = (uint64_t)jobs[i].n_rows * (uint64_t)jobs[i].n_cols;
  const std::vector<int> order = order_by_falling(work);
  // pass 1: a small job's XCD, or a large job's XCD order (3 bits each)
  std::vector<uint32_t> where(nj);
  int64_t load[X] = {0};
  int64_t cnt[X] = {0};
  for (int j : order) {
    const KnnJob &J = jobs[(size_t)j];
    const int64_t nrb = (J.n_rows + rpi - 1) / rpi;
    const int64_t w_item = rpi * (int64_t)J.n_cols;
    if (nrb <= 16) {
      int x = 0;
      for (int y = 1; y < X; ++y)
        if (load[y] < load[x]) x = y;
      where[(size_t)j] = (uint32_t)x;
      load[x] += w_item * nrb;
      cnt[x] += nrb;
    } else {
      int rank[X];
      for (int q = 0; q < X; ++q) {  // XCDs by rising load (stable insertion)
        int p = q;
        while (p > 0 && load[rank[p - 1]] > load[q]) {
          rank[p] = rank[p - 1];
          --p;
        }
        rank[p] = q;
      }
      uint32_t code = 0;
      for (int q = 0; q < X; ++q) {
        const int64_t c = nrb / X + (q < nrb % X ? 1 : 0);
        load[rank[q]] += w_item * c;
        cnt[rank[q]] += c;
        code |= (uint32_t)rank[q] << (3 * q);
      }
      where[(size_t)j] = code;
    }
  }
  int64_t mx = 0;
  for (int x = 0; x < X; ++x) mx = std::max(mx, cnt[x]);
  std::vector<KnnItem> items((size_t)(mx * X));
  // pass 2: the items in place
  int64_t cur[X] = {0};
  for (int j : order) {
    const KnnJob &J = jobs[(size_t)j];
    const int nrb = (int)((J.n_rows + rpi - 1) / rpi);
    const uint32_t w = where[(size_t)j];
    if (nrb <= 16) {
      const int x = (int)w;
      for (int rb = 0; rb < nrb; ++rb) items[(size_t)((cur[x] + rb) * X + x)] = KnnItem{j, rb};
      cur[x] += nrb;
    } else {
      for (int rb = 0; rb < nrb; ++rb) {
        const int x = (int)((w >> (3 * (rb % X))) & 7u);
        items[(size_t)(cur[x]++ * X + x)] = KnnItem{j, rb};
      }
    }
  }
  for (int x = 0; x < X; ++x)
    for (int64_t i = cur[x]; i < mx; ++i) items[(size_t)(i * X + x)] = KnnItem{-1, 0};
  return items;
}

}  // namespace

namespace {

// Scratch of pipnn_hashprune_insert_static: one array per device, held from
// the library's load until the process ends. Host code never passes the
// array's name to a kernel (on the host it is a stand-in symbol, not a
// device address); static_scratch() looks up its address on each device
// once, with that device current, and the kernels get that pointer.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kMaxDevices] = {};

hipError_t static_scratch(int dev, unsigned char **out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<unsigned char *>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

namespace pipnn {

hipError_t DevBuf::ensure(size_t bytes) {
  if (bytes <= cap && p) return hipSuccess;
  if (fixed) {
    // a slice of the caller's workspace: handed out whole on first use
    if (bytes > lim || !ws_p) return hipErrorOutOfMemory;
    p = ws_p;
    cap = lim;
    return hipSuccess;
  }
  // a buffer that has to grow again takes half as much once more, so that
  // calls of slowly rising size (insertions) reallocate rarely
  const size_t grown = p ? cap + cap / 2 : 0;
  release();
  const size_t want = std::max<size_t>({bytes, grown, (size_t)256});
  hipError_t e = hipMalloc(&p, want);
  if (e != hipSuccess) {
    p = nullptr;
    cap = 0;
    return e;
  }
  cap = want;
  return hipSuccess;
}

hipError_t HostStage::put(DevBuf &dst, const void *src, size_t bytes, hipStream_t s) {
  hipError_t e = dst.ensure(std::max<size_t>(bytes, 1));
  if (e != hipSuccess || bytes == 0) return e;
  const size_t need = (bytes + 255) & ~(size_t)255;
  if (used + need > cap) {
    // the pending copies read the buffer: wait for them, then start over
    if (used > 0 && (e = hipStreamSynchronize(s)) != hipSuccess) return e;
    used = 0;
    if (need > cap) {
      release();
      const size_t want = std::max<size_t>(need, (size_t)1 << 20);
      if ((e = hipHostMalloc(reinterpret_cast<void **>(&p), want)) != hipSuccess) {
        p = nullptr;
        return e;
      }
      cap = want;
    }
  }
  memcpy(p + used, src, bytes);
  e = hipMemcpyAsync(dst.p, p + used, bytes, hipMemcpyHostToDevice, s);
  used += need;
  return e;
}

void HostStage::release() {
  if (p) (void)hipHostFree(p);
  p = nullptr;
  cap = used = 0;
}

void DevBuf::release() {
  if (p && !fixed) (void)hipFree(p);
  p = nullptr;
  cap = 0;
}

const float *Index::xf() const {
  return x_dtype == PIPNN_DTYPE_F32 ? reinterpret_cast<const float *>(X) : xf32.as<float>();
}

const float *Index::xop32() const { return xpad.p ? xpad.as<float>() : xf(); }

static hipEvent_t take_event(Index &I) {
  if (!I.ev_free.empty()) {
    hipEvent_t e = I.ev_free.back();
    I.ev_free.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

PhaseTimer::PhaseTimer(Index &I_, int ph, hipStream_t s_) : I(I_), phase(ph), s(s_) {
  if (!I.profiling || stream_capturing(s)) return;
  a = take_event(I);
  if (a) (void)hipEventRecord(a, s);
}

PhaseTimer::~PhaseTimer() {
  if (!a) return;
  hipEvent_t b = take_event(I);
  if (!b) {
    I.ev_free.push_back(a);
    return;
  }
  (void)hipEventRecord(b, s);
  I.events.push_back({phase, a, b});
}

// Flush recorded event pairs into the per-phase sums.
static void flush_events(Index &I) {
  for (auto &e : I.events) {
    float ms = 0.f;
    if (hipEventSynchronize(e.b) == hipSuccess && hipEventElapsedTime(&ms, e.a, e.b) == hipSuccess)
      I.phase_ms[e.phase] += ms;
    I.ev_free.push_back(e.a);
    I.ev_free.push_back(e.b);
  }
  I.events.clear();
}

}  // namespace pipnn

namespace {

// The fp16 copy of a float32 index of at most 128 dimensions, kept while X
// is integral (int_exact): made or refreshed by create and prepare; outside
// stream capture it also reads back whether the copy holds X exactly. Where
// it does, the partition's leader distances and RobustPrune's rows come from
// it (half the bytes, the same values; every distance form is the same
// integer in either format).
hipError_t refresh_fp32_copy(Index &I, hipStream_t s) {
  if (I.p.gemm_prec != PIPNN_PREC_FP32 || I.d > 128) return hipSuccess;
  const bool capturing = stream_capturing(s);
  if (!I.int_exact) {
    if (!capturing) I.op_exact = false;
    I.i8_ok = false;
    return hipSuccess;
  }
  hipError_t e;
  if (!I.xlow.p) {
    if (capturing) return hipSuccess;  // no copy yet: op_exact stays false
    I.copy_prec = PIPNN_PREC_FP16;
    I.ldo = lowp_padded_dim(I.d);
    const size_t c = (size_t)I.cap;
    if ((e = I.xlow.ensure(c * I.ldo * 2)) != hipSuccess ||
        (e = I.xscale.ensure(c * 4)) != hipSuccess || (e = I.lnorms.ensure(c * 4)) != hipSuccess ||
        (e = I.op_flag.ensure(64)) != hipSuccess)
      return e;
  }
  // the int8 rows (L2): coordinates of range <= 255 fit int8 after the shift
  I.i8_ok = false;
  const bool with8 =
      I.p.metric == PIPNN_METRIC_L2 && I.int_hi - I.int_lo <= 255 && (I.x8.p || !capturing);
  if (with8) {
    I.ld8 = rows8_width(I.d);
    const size_t c = (size_t)I.cap;
    if ((e = I.x8.ensure(c * I.ld8)) != hipSuccess || (e = I.n8.ensure(c * 4)) != hipSuccess)
      return e;
    I.lo8 = I.int_lo;
  }
  if ((e = clear_op_flag(I, s)) != hipSuccess ||
      (e = launch_quantize_range(I, 0, I.n, s, with8)) != hipSuccess)
    return e;
  I.i8_ok = with8;
  return capturing ? hipSuccess : read_op_flag(I, true, s);
}

// The int8 rows of an index whose GEMM operand is a reduced-precision copy
// (the float32 index makes them with its fp16 copy, above): kept while X is
// integral and spans at most 256 values (L2, d <= 128).
hipError_t refresh_rows8(Index &I, hipStream_t s) {
  const bool capturing = stream_capturing(s);
  const bool want = I.p.metric == PIPNN_METRIC_L2 && I.d <= 128 && I.int_exact &&
                    I.int_hi - I.int_lo <= 255 && (I.x8.p || !capturing);
  I.i8_ok = false;
  if (!want) return hipSuccess;
  I.ld8 = rows8_width(I.d);
  const size_t c = (size_t)I.cap;
  hipError_t e;
  if ((e = I.x8.ensure(c * I.ld8)) != hipSuccess || (e = I.n8.ensure(c * 4)) != hipSuccess)
    return e;
  I.lo8 = I.int_lo;
  if ((e = launch_quantize8_range(I, 0, I.n, s)) != hipSuccess) return e;
  I.i8_ok = true;
  return hipSuccess;
}

// ---------------------------------------------------------------------
// Workspace layout. Every device buffer of an index has a worst-case size
// that follows from the parameters, n, d, the dtype of X and the leaf rows
// of one pick + binning batch. On a caller's workspace each buffer is a
// fixed slice of that size (256-byte aligned, in the order of all_bufs), so
// pipnn_workspace_bytes is the sum of the slices and nothing is allocated.
//
// The partition bounds follow from Alg. 5 with fanout: a point is assigned
// to at most fanout[l] leaders at level l, so the subproblems of any level
// hold at most F = n * fanout[0] * fanout[1] * fanout[2] members (fanout[3]
// is 1), their assignments at most F, and the leaves of one partition at
// most F members in total; every subproblem below the root has more than
// C_max members, and a subproblem of c members has at most
// min(leader_cap, c / leader_div + 3) leaders (buckets).

constexpr int64_t kMaxLeafRows = 65535;       // the largest leaf a build takes
constexpr int64_t kMaxBatchRows = (int64_t)1 << 25;
constexpr int64_t kSeenBudgetWords = (int64_t)1 << 26;  // 256 MiB of search seen-bitmaps
constexpr int64_t kMaxQueryBatch = (int64_t)1 << 16;
constexpr int64_t kGraphMaxK1 = 65;           // k + 1 of a full k-NN graph chunk
constexpr int64_t kA2aBudgetFloats = (int64_t)1 << 28;  // all-to-all distance matrices of a batch

int64_t members_bound(const pipnn_params &p, int64_t n) {
  return n * p.fanout[0] * p.fanout[1] * p.fanout[2];
}

// Leaf rows of one batch for max_batch_records records (a pick gives two):
// at least the largest leaf, at most a whole build. 0: a whole build.
int64_t batch_rows_for(const pipnn_params &p, int64_t n, int64_t max_batch_records) {
  const int64_t whole =
      std::min<int64_t>(kMaxBatchRows, std::max<int64_t>(kMaxLeafRows, members_bound(p, n)));
  if (max_batch_records <= 0) return whole;
  return std::max<int64_t>(kMaxLeafRows,
                           std::min<int64_t>(whole, max_batch_records / (2 * (int64_t)p.k)));
}

// Queries per search launch (their seen bitmaps take n bits each).
int64_t query_batch(int64_t n) {
  const int64_t words = (n + 31) / 32;
  return std::max<int64_t>(1, std::min<int64_t>(kMaxQueryBatch, kSeenBudgetWords / words));
}

// The shape-dependent fields of an index (also set on a host-only index by
// pipnn_workspace_bytes).
void init_shape(Index &I, const pipnn_params &p, int64_t n, int32_t d, int32_t x_dtype) {
  I.p = p;
  I.n = n;
  I.cap = n;
  I.d = d;
  I.x_dtype = x_dtype;
  I.m = p.hash_bits;
  I.ldf = knn_operand_dim(d, PIPNN_PREC_FP32);
}

std::vector<DevBuf *> all_bufs(Index &I) {
  return {&I.flag, &I.int_chk, &I.op_flag, &I.s_counter, &I.sketches, &I.norms, &I.xf32,
          &I.xpad, &I.xlow, &I.xscale, &I.lnorms, &I.rp_order, &I.lt_off, &I.lt_mem, &I.lt_rep,
          &I.s_jobs, &I.s_items, &I.s_picks_c, &I.s_picks_d, &I.s_cnt, &I.s_off, &I.s_bins,
          &I.s_tmp0, &I.s_tmp1, &I.p_mem[0], &I.p_mem[1], &I.p_asg, &I.p_G, &I.p_gout,
          &I.p_gsize, &I.p_leaders, &I.p_cm, &I.p_bstart, &I.p_groups, &I.p_seg, &I.p_seglen,
          &I.p_segfirst, &I.p_segoff, &I.p_rsrc, &I.p_roff, &I.p_rlen, &I.p_esrc, &I.p_eoff,
          &I.p_elen, &I.o_first, &I.o_flag, &I.o_pos, &I.o_pos2, &I.o_tmp, &I.plan.jobs,
          &I.plan.items, &I.i_rows, &I.i_cols, &I.i_assign, &I.i_flag, &I.i_pos, &I.i_list,
          &I.i_tmp, &I.i_segs, &I.q_conv, &I.q_seen, &I.g_ids, &I.g_dist, &I.a2a_mat,
          &I.a2a_tmp, &I.x8, &I.n8};
}

size_t slice_bytes(size_t b) { return (std::max<size_t>(b, 256) + 255) & ~(size_t)255; }

// Sets every buffer's lim for the index's shape and batch_rows. Buffers
// only insertion uses get none (an index on a workspace holds a fixed set of
// points).
void set_limits(Index &I) {
  const pipnn_params &P = I.p;
  const int64_t n = I.n, d = I.d, k = P.k, B = I.batch_rows;
  const int64_t F = std::max<int64_t>(n, members_bound(P, n));
  const int64_t S = std::max<int64_t>(1, F / ((int64_t)P.c_max + 1));      // subproblems per level
  const int64_t ell_max = std::min<int64_t>(P.leader_cap, F / P.leader_div + 3);
  // (each bound adds one per subproblem and one more for integer division)
  const int64_t NB = F / P.leader_div + 3 * S + 1;                          // buckets per level
  const int64_t tiles = F / kGroupTile + S + 1;                             // group-by tiles
  const int64_t CM = ell_max * tiles;                                       // group-by counters
  const int64_t LV = 2 * NB + F / P.c_max + S + 1;                          // leaves per level
  const int64_t mx = std::max(F, n);
  const size_t nb_start = (size_t)((n + 255) / 256);
  for (DevBuf *b : all_bufs(I)) b->lim = 0;
  I.flag.lim = I.int_chk.lim = I.op_flag.lim = I.s_counter.lim = 64;
  I.sketches.lim = (size_t)n * I.m * 4;
  I.norms.lim = (size_t)n * 4;
  if (I.x_dtype != PIPNN_DTYPE_F32) I.xf32.lim = (size_t)n * d * 4;
  if (I.ldf != 0 && I.ldf != d) I.xpad.lim = (size_t)n * I.ldf * 4;
  if (P.gemm_prec != PIPNN_PREC_FP32 || d <= 128) {
    const size_t eb = P.gemm_prec == PIPNN_PREC_FP8 ? 1 : 2;
    I.xlow.lim = (size_t)n * lowp_padded_dim((int)d) * eb;
    I.xscale.lim = I.lnorms.lim = (size_t)n * 4;
  }
  if (d <= 128 && P.metric == PIPNN_METRIC_L2) {
    I.x8.lim = (size_t)n * rows8_width((int)d);
    I.n8.lim = (size_t)n * 4;
  }
  I.rp_order.lim = (size_t)n * 4;
  I.lt_off.lim = (size_t)(F + 1) * 8;
  I.lt_mem.lim = (size_t)F * 4;
  // work lists: a partition level (its subproblems, row blocks of 128), or
  // a batch of leaves (a job per leaf of two or more rows, row blocks of at
  // least 32), or one block
  const int64_t jobs = std::max<int64_t>(S, B / 2 + 1);
  const int64_t items = std::max<int64_t>(F / 128 + S + 1, B / 32 + B / 2 + 2);
  I.s_jobs.lim = (size_t)jobs * sizeof(KnnJob);
  I.s_items.lim = (size_t)items * sizeof(KnnItem);
  I.s_picks_c.lim = I.s_picks_d.lim = (size_t)B * k * 4;
  I.s_bins.lim = (size_t)2 * B * k * 8;
  I.s_cnt.lim = (size_t)n * 4;
  I.s_off.lim = std::max<size_t>((size_t)(n + 1) * 8, (size_t)scan_tmp_elems(CM) * 8);
  I.s_tmp0.lim = std::max<size_t>((size_t)scan_tmp_elems(n) * 8, (size_t)S * sizeof(GroupSub));
  I.s_tmp1.lim = std::max<size_t>((size_t)NB * 8, ((size_t)d + 2 * nb_start + 1) * 8 + 8);
  I.p_mem[0].lim = I.p_mem[1].lim = I.p_asg.lim = I.p_G.lim = I.p_gout.lim = (size_t)F * 4;
  I.p_gsize.lim = I.p_leaders.lim = I.p_seglen.lim = I.p_rlen.lim = (size_t)NB * 4;
  I.p_segfirst.lim = (size_t)(NB + 1) * 4;
  I.p_seg.lim = I.p_segoff.lim = I.p_rsrc.lim = I.p_roff.lim = (size_t)NB * 8;
  I.p_bstart.lim = (size_t)(NB + 1) * 8;
  I.p_cm.lim = (size_t)(CM + 1) * 8;
  I.p_groups.lim = (size_t)tiles * sizeof(GroupTile);
  I.p_esrc.lim = I.p_eoff.lim = (size_t)LV * 8;
  I.p_elen.lim = (size_t)LV * 4;
  I.o_first.lim = (size_t)n * 4;
  I.o_flag.lim = (size_t)mx * 4;
  I.o_pos.lim = (size_t)(mx + 1) * 8;
  I.o_pos2.lim = (size_t)(n + 1) * 8;
  I.o_tmp.lim = (size_t)scan_tmp_elems(mx) * 8;
  // a planned build: every batch's jobs and row blocks
  I.plan.jobs.lim = (size_t)(F / 2 + F / B + 2) * sizeof(KnnJob);
  I.plan.items.lim = (size_t)(F / 32 + F / 2 + F / B + 2) * sizeof(KnnItem);
  const int64_t QB = query_batch(n);
  I.q_conv.lim = (size_t)QB * d * 4;
  I.q_seen.lim = (size_t)QB * ((n + 31) / 32) * 4;
  I.g_ids.lim = I.g_dist.lim = (size_t)std::min<int64_t>(n, QB) * kGraphMaxK1 * 4;
  if (P.leaf_picker == PIPNN_PICKER_ALL_TO_ALL) {
    I.a2a_mat.lim = (size_t)kA2aBudgetFloats * 4;
    I.a2a_tmp.lim = (size_t)B * 8;
  }
}

// Sum of the slices of the layout.
size_t layout_bytes(Index &I) {
  size_t t = 0;
  for (DevBuf *b : all_bufs(I))
    if (b->lim) t += slice_bytes(b->lim);
  return t;
}

}  // namespace

// All-to-All Prune leaf picker: batches of leaves whose distance matrices
// (rows x largest leaf x 4 B) fit 1 GiB.
std::vector<std::pair<int64_t, int64_t>> a2a_batches(const std::vector<int64_t> &offs,
                                                     int64_t l0, int64_t l1) {
  const int64_t budget = kA2aBudgetFloats;
  std::vector<std::pair<int64_t, int64_t>> out;
  int64_t b0 = l0, rows = 0, wide = 1;
  for (int64_t l = l0; l < l1; ++l) {
    const int64_t sz = offs[(size_t)l + 1] - offs[(size_t)l];
    const int64_t w2 = std::max(wide, sz);
    if (l > b0 && (rows + sz) * w2 > budget) {
      out.push_back({b0, l});
      b0 = l;
      rows = 0;
      wide = 1;
    }
    rows += sz;
    wide = std::max(wide, sz);
  }
  if (b0 < l1) out.push_back({b0, l1});
  return out;
}

extern "C" {

const char *pipnn_version(void) { return "pipnn-gfx950 0.1.0"; }

const char *pipnn_last_error(void) { return g_err.c_str(); }

void pipnn_default_params(pipnn_params *p) {
  if (!p) return;
  memset(p, 0, sizeof(*p));
  p->metric = PIPNN_METRIC_L2;
  p->c_max = 1024;
  p->c_min = 64;
  p->leader_div = 200;
  p->leader_cap = 1000;
  p->fanout[0] = 2;
  p->fanout[1] = p->fanout[2] = p->fanout[3] = 1;
  p->k = 16;
  p->hash_bits = 12;
  p->l_max = 64;
  p->R = 32;
  p->alpha = 1.2f;
  p->gemm_prec = PIPNN_PREC_FP32;
  p->rescore_mult = 0;
  p->rescore_extra = 0;
  p->seed = 0;
}

size_t pipnn_workspace_bytes(const pipnn_params *p, int64_t n, int32_t d, int32_t x_dtype,
                             int64_t max_batch_records) {
  try {
    std::string why;
    if (!valid_params(p, why) || n < 2 || n >= (int64_t)0xFFFFFFFFll || d < 1 || d > 1024)
      return 0;
    if (x_dtype != PIPNN_DTYPE_F32 && x_dtype != PIPNN_DTYPE_F16 && x_dtype != PIPNN_DTYPE_BF16)
      return 0;
    Index I;
    init_shape(I, *p, n, d, x_dtype);
    I.batch_rows = batch_rows_for(*p, n, max_batch_records);
    set_limits(I);
    return layout_bytes(I);
  } catch (...) {
    return 0;
  }
}

pipnn_status pipnn_create(const pipnn_params *p, const void *d_X, int64_t n, int32_t d,
                          int32_t x_dtype, const float *d_H, void *d_workspace, size_t ws_bytes,
                          pipnn_stream_t stream, pipnn_index **out) {
  GUARD_BEGIN
  std::string why;
  if (!out) return fail(PIPNN_EINVAL, "out is NULL");
  *out = nullptr;
  if (!valid_params(p, why)) return fail(PIPNN_EINVAL, "invalid params: %s", why.c_str());
  if (!d_X || !d_H) return fail(PIPNN_EINVAL, "X or H is NULL");
  if (n < 2 || n >= (int64_t)0xFFFFFFFFll) return fail(PIPNN_EINVAL, "n must be in 2..2^32-2");
  if (d < 1 || d > 1024) return fail(PIPNN_EINVAL, "d must be in 1..1024");
  if (x_dtype != PIPNN_DTYPE_F32 && x_dtype != PIPNN_DTYPE_F16 && x_dtype != PIPNN_DTYPE_BF16)
    return fail(PIPNN_EINVAL, "unknown x_dtype %d", x_dtype);
  const bool ws = d_workspace != nullptr || ws_bytes != 0;
  if (ws) {
    if (!d_workspace) return fail(PIPNN_EINVAL, "workspace is NULL but ws_bytes is not 0");
    if (reinterpret_cast<uintptr_t>(d_workspace) & 255u)
      return fail(PIPNN_EINVAL, "the workspace must be 256-byte aligned");
    if (x_dtype == PIPNN_DTYPE_F32 && (reinterpret_cast<uintptr_t>(d_X) & 15u))
      return fail(PIPNN_EINVAL, "an index on a workspace needs a 16-byte aligned float32 X");
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  Index *I = new Index();
  init_shape(*I, *p, n, d, x_dtype);
  I->X = d_X;
  I->H = d_H;
  I->stream = s;
  auto cleanup = [&](pipnn_status st) {
    pipnn_destroy(reinterpret_cast<pipnn_index *>(I));
    return st;
  };
  if (ws) {
    // the largest batch of leaf rows whose layout fits the workspace
    auto bytes_at = [&](int64_t rows) {
      I->batch_rows = rows;
      set_limits(*I);
      return layout_bytes(*I);
    };
    int64_t lo = kMaxLeafRows, hi = batch_rows_for(*p, n, 0);
    const size_t need_min = bytes_at(lo);
    if (need_min > ws_bytes)
      return cleanup(fail(PIPNN_ENOMEM, "the workspace has %zu bytes; this index needs at least "
                          "%zu (pipnn_workspace_bytes)", ws_bytes, need_min));
    if (bytes_at(hi) > ws_bytes) {
      while (lo < hi) {  // bytes_at(lo) fits, bytes_at(hi) does not
        const int64_t mid = lo + (hi - lo + 1) / 2;
        if (bytes_at(mid) <= ws_bytes) lo = mid; else hi = mid - 1;
      }
    } else {
      lo = hi;
    }
    I->ws_bytes = bytes_at(lo);
    unsigned char *base = static_cast<unsigned char *>(d_workspace);
    size_t off = 0;
    for (DevBuf *b : all_bufs(*I)) {
      b->fixed = true;
      if (!b->lim) continue;
      b->ws_p = base + off;
      off += slice_bytes(b->lim);
    }
    I->ws_mode = true;
  }
  hipError_t e;
  {
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) == hipSuccess) I->device = dev;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        ncu >= kNumXcd)
      I->n_cu = ncu;
  }
  I->cap = n;
  // leaf-kernel default: four lanes per row where that layout is built for
  // the operand, except fp8 (two lanes); pipnn_autotune may change it. Four
  // lanes hold a row's kept list in a quarter of the registers each, so an
  // insertion compares fewer keys per lane: on 1M points of 128 (96) dims
  // the bf16 pick took 2.55 ms against 2.68 ms (two lanes) for k = 16 and
  // 6.9 (7.1) ms against 7.5 (8.9) ms with 32 selected for rescoring.
  I->leaf_quad = (p->gemm_prec != PIPNN_PREC_FP8 && knn_quad_available(d, p->gemm_prec)) ? 1 : 0;
  if (p->gemm_prec == PIPNN_PREC_FP32 && knn_operand_dim(d, PIPNN_PREC_FP32) == 0)
    return cleanup(fail(PIPNN_EINVAL, "a float32 leaf GEMM needs d <= 256 (use a reduced "
                                      "gemm_prec for wider vectors)"));
  if ((e = I->s_counter.ensure(64)) != hipSuccess ||
      (e = I->sketches.ensure((size_t)n * I->m * 4)) != hipSuccess ||
      (e = I->norms.ensure((size_t)n * 4)) != hipSuccess ||
      (e = I->int_chk.ensure(64)) != hipSuccess ||
      (e = I->flag.ensure(64)) != hipSuccess)
    return cleanup(fail(PIPNN_ENOMEM, "device allocation failed: %s", hipGetErrorString(e)));
  if (x_dtype != PIPNN_DTYPE_F32) {
    if ((e = I->xf32.ensure((size_t)n * d * 4)) != hipSuccess)
      return cleanup(fail(PIPNN_ENOMEM, "device allocation failed: %s", hipGetErrorString(e)));
    if ((e = launch_to_f32(d_X, x_dtype, I->xf32.as<float>(), n * (int64_t)d, s)) != hipSuccess)
      return cleanup(fail(PIPNN_EDEVICE, "conversion launch failed: %s", hipGetErrorString(e)));
  }
  if ((e = clear_int_check(*I, s)) != hipSuccess || (e = launch_norms_sketches(*I, s)) != hipSuccess ||
      (e = read_int_check(*I, true, s)) != hipSuccess)
    return cleanup(fail(PIPNN_EDEVICE, "sketch launch failed: %s", hipGetErrorString(e)));
  // the float32 GEMM operand: X itself when its rows are whole 16-byte
  // vectors of an instantiated width, else a zero-padded copy
  I->ldf = knn_operand_dim(d, PIPNN_PREC_FP32);
  if (I->ldf != 0 && (I->ldf != d || (reinterpret_cast<uintptr_t>(I->xf()) & 15u) != 0)) {
    if ((e = I->xpad.ensure((size_t)n * I->ldf * 4)) != hipSuccess)
      return cleanup(fail(PIPNN_ENOMEM, "device allocation failed: %s", hipGetErrorString(e)));
    if ((e = launch_pad_range(*I, 0, n, s)) != hipSuccess)
      return cleanup(fail(PIPNN_EDEVICE, "pad launch failed: %s", hipGetErrorString(e)));
  }
  if ((e = refresh_fp32_copy(*I, s)) != hipSuccess)
    return cleanup(fail(e == hipErrorOutOfMemory ? PIPNN_ENOMEM : PIPNN_EDEVICE,
                        "fp16 copy failed: %s", hipGetErrorString(e)));
  if (p->gemm_prec != PIPNN_PREC_FP32) {
    I->copy_prec = p->gemm_prec;
    I->ldo = lowp_padded_dim(d);
    if (I->ldo == 0)
      return cleanup(fail(PIPNN_EINVAL, "a reduced-precision leaf GEMM needs d <= 768"));
    const size_t eb = p->gemm_prec == PIPNN_PREC_FP8 ? 1 : 2;
    if ((e = I->xlow.ensure((size_t)n * I->ldo * eb)) != hipSuccess ||
        (e = I->xscale.ensure((size_t)n * 4)) != hipSuccess ||
        (e = I->lnorms.ensure((size_t)n * 4)) != hipSuccess ||
        (e = I->op_flag.ensure(64)) != hipSuccess)
      return cleanup(fail(PIPNN_ENOMEM, "device allocation failed: %s", hipGetErrorString(e)));
    if ((e = clear_op_flag(*I, s)) != hipSuccess || (e = launch_quantize(*I, s)) != hipSuccess ||
        (e = read_op_flag(*I, true, s)) != hipSuccess)
      return cleanup(fail(PIPNN_EDEVICE, "quantize launch failed: %s", hipGetErrorString(e)));
    if ((e = refresh_rows8(*I, s)) != hipSuccess)
      return cleanup(fail(e == hipErrorOutOfMemory ? PIPNN_ENOMEM : PIPNN_EDEVICE,
                          "int8 rows failed: %s", hipGetErrorString(e)));
  }
  if ((e = hipMemsetAsync(I->flag.p, 0, 64, s)) != hipSuccess)
    return cleanup(fail(PIPNN_EDEVICE, "memset failed: %s", hipGetErrorString(e)));
  *out = reinterpret_cast<pipnn_index *>(I);
  return PIPNN_OK;
  GUARD_END
}

void pipnn_destroy(pipnn_index *idx) {
  if (!idx) return;
  Index *I = reinterpret_cast<Index *>(idx);
  // the caller has finished the work that uses the index (no device-wide
  // synchronisation: other streams keep running); hipFree waits for the
  // device where it must
  for (DevBuf *b : all_bufs(*I)) b->release();
  I->stage.release();
  for (auto &e : I->events) {
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  for (hipEvent_t e : I->ev_free) (void)hipEventDestroy(e);
  delete I;
}

// ---------------------------------------------------------------------
// Randomized ball carving (Alg. 5), level by level.
pipnn_status pipnn_partition(pipnn_index *idx, int64_t *d_leaf_offsets, int64_t cap_leaves,
                             uint32_t *d_leaf_members, int64_t cap_members, int64_t *h_n_leaves,
                             int64_t *h_n_members, pipnn_stream_t stream) {
  return pipnn_partition_replica(idx, 0, d_leaf_offsets, cap_leaves, d_leaf_members, cap_members,
                                 h_n_leaves, h_n_members, stream);
}

pipnn_status pipnn_partition_replica(pipnn_index *idx, int32_t replica, int64_t *d_leaf_offsets,
                                     int64_t cap_leaves, uint32_t *d_leaf_members,
                                     int64_t cap_members, int64_t *h_n_leaves,
                                     int64_t *h_n_members, pipnn_stream_t stream) {
  GUARD_BEGIN
  if (!idx || !h_n_leaves || !h_n_members) return fail(PIPNN_EINVAL, "NULL argument");
  if (replica < 0) return fail(PIPNN_EINVAL, "replica must be >= 0");
  Index &I = *reinterpret_cast<Index *>(idx);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const pipnn_params &P = I.p;
  const int64_t n = I.n;
  // point-to-leader distances on the index's reduced-precision operand when
  // it holds X exactly or the float32 kernel is not built (d > 256), else
  // in float32
  int32_t part_prec = PIPNN_PREC_FP32;
  if (P.gemm_prec == PIPNN_PREC_FP32)
    part_prec = I.copy16_exact() ? I.copy_prec : PIPNN_PREC_FP32;
  else if (I.op_exact || !knn_operand_dim(I.d, PIPNN_PREC_FP32))
    part_prec = P.gemm_prec;
  if (knn_operand_dim(I.d, part_prec) == 0)
    return fail(PIPNN_EINVAL, "partition of d = %d needs a reduced gemm_prec (float32 partition "
                              "distances are built for d <= 256)", I.d);

  struct Sub {
    int64_t row_off, cnt;
    uint64_t key;
    int depth;
  };
  // Leaves are written to the output level by level, in the order they are
  // found, so that one level's buffers serve the next: the members of the
  // level's subproblems (ping-pong between p_mem[0] and p_mem[1]), their
  // leader assignments (p_asg), the assignments grouped by bucket (p_G) and
  // the merged small buckets (p_gout).
  struct Leaf {
    const uint32_t *src;
    int64_t len;  // -1: the size of merged group `grp`, read back
    int32_t grp;
  };
  std::vector<int64_t> offs(1, 0);  // output CSR offsets (host)
  bool writing = d_leaf_offsets && d_leaf_members;
  PhaseTimer timer(I, kPhPartition, s);
  int64_t leader_dists = 0;
  int levels = 0;
  // appends a level's leaves; members are copied while everything so far
  // fits the output's capacities
  auto emit = [&](const std::vector<Leaf> &lv, const std::vector<int32_t> &grp_size) -> pipnn_status {
    if (lv.empty()) return PIPNN_OK;
    const int64_t base = offs.back();
    std::vector<const uint32_t *> src;
    std::vector<int64_t> doff;
    std::vector<int32_t> lens;
    for (const Leaf &lf : lv) {
      const int64_t len = lf.len >= 0 ? lf.len : grp_size[(size_t)lf.grp];
      src.push_back(lf.src);
      doff.push_back(offs.back() - base);
      lens.push_back((int32_t)len);
      offs.push_back(offs.back() + len);
    }
    if ((int64_t)offs.size() - 1 > cap_leaves || offs.back() > cap_members) writing = false;
    if (!writing) return PIPNN_OK;
    HIPCHK(staged(I, I.p_esrc, src, s));
    HIPCHK(staged(I, I.p_eoff, doff, s));
    HIPCHK(staged(I, I.p_elen, lens, s));
    HIPCHK(launch_copy_segments(I.p_esrc.as<const uint32_t *>(), I.p_eoff.as<int64_t>(),
                                I.p_elen.as<int32_t>(), (int32_t)src.size(),
                                d_leaf_members + base, s));
    return PIPNN_OK;
  };

  int cur = 0;
  HIPCHK(I.p_mem[0].ensure((size_t)n * 4));
  HIPCHK(launch_iota(I.p_mem[0].as<uint32_t>(), n, s));
  std::vector<Sub> subs;
  if (n <= P.c_max) {
    pipnn_status st = emit({{I.p_mem[0].as<uint32_t>(), n, 0}}, {});
    if (st != PIPNN_OK) return st;
  } else {
    subs.push_back({0, n, replica_key(P.seed, replica), 0});
  }

  while (!subs.empty()) {
    const uint32_t *A = I.p_mem[cur].as<uint32_t>();
    // --- leaders and assignment jobs
    std::vector<KnnJob> jobs;
    std::vector<KnnItem> items;
    std::vector<int64_t> lead_idx;
    std::vector<int32_t> ells, fs;
    int64_t inst = 0;
    int fmax = 1;
    for (size_t si = 0; si < subs.size(); ++si) {
      const Sub &sb = subs[si];
      int64_t ell = (sb.cnt + P.leader_div - 1) / P.leader_div;
      ell = std::max<int64_t>(ell, 2);
      ell = std::min<int64_t>(ell, P.leader_cap);
      ell = std::min<int64_t>(ell, sb.cnt);
      int f = P.fanout[std::min(sb.depth, 3)];
      f = (int)std::min<int64_t>(f, ell);
      f = std::max(f, 1);
      fmax = std::max(fmax, f);
      const int64_t lead_off = (int64_t)lead_idx.size();
      for (int64_t pos : leader_positions(sb.key, sb.cnt, ell)) lead_idx.push_back(sb.row_off + pos);
      KnnJob J{};
      J.row_off = sb.row_off;
      J.col_off = lead_off;
      J.out_off = sb.row_off;
      J.n_rows = (int32_t)sb.cnt;
      J.n_cols = (int32_t)ell;
      J.k_sel = f;
      J.flags = 0;
      jobs.push_back(J);
      ells.push_back((int32_t)ell);
      fs.push_back(f);
      inst += sb.cnt;
      leader_dists += sb.cnt * ell;
    }
    ++levels;
    HIPCHK(staged(I, I.s_tmp1, lead_idx, s));
    HIPCHK(I.p_leaders.ensure(lead_idx.size() * 4));
    HIPCHK(launch_gather_u32(A, I.s_tmp1.as<int64_t>(), I.p_leaders.as<uint32_t>(),
                             (int64_t)lead_idx.size(), s));
    items = plan_items(jobs, 128);
    HIPCHK(staged(I, I.s_jobs, jobs, s));
    HIPCHK(staged(I, I.s_items, items, s));
    HIPCHK(I.p_asg.ensure((size_t)inst * fmax * 4));
    KnnLaunch L{};
    L.idx = &I;
    L.row_base = A;
    L.col_base = I.p_leaders.as<uint32_t>();
    L.jobs = I.s_jobs.as<KnnJob>();
    L.items = I.s_items.as<KnnItem>();
    L.n_items = (int32_t)items.size();
    L.ksel = fmax;
    L.k_out = fmax;
    L.out_ids = 0;
    L.recompute = 0;
    L.rescore_k = 0;
    L.prec = part_prec;
    L.nw = 4;
    L.persistent = 0;
    // float32 leader distances in the four-lane layout (where built), the
    // reduced-precision ones in the two-lane layout
    L.quad = knn_quad_available(I.d, part_prec) ? 1 : 0;
    L.out_col = I.p_asg.as<uint32_t>();
    L.out_dist = nullptr;
    L.out_matrix = nullptr;
    HIPCHK(launch_knn(L, s));

    // --- stable group-by into buckets
    std::vector<GroupSub> gsubs;
    std::vector<GroupTile> tiles;
    std::vector<int64_t> bucket_cm;
    int64_t cm_len = 0, nbuck = 0;
    for (size_t si = 0; si < subs.size(); ++si) {
      GroupSub g;
      g.elem_off = subs[si].row_off * fmax;
      g.n_elems = subs[si].cnt * fmax;
      g.n_buckets = ells[si];
      g.n_tiles = (int32_t)((g.n_elems + kGroupTile - 1) / kGroupTile);
      g.cm_off = cm_len;
      g.bucket_off = nbuck;
      for (int t = 0; t < g.n_buckets; ++t) bucket_cm.push_back(g.cm_off + (int64_t)t * g.n_tiles);
      for (int t = 0; t < g.n_tiles; ++t) tiles.push_back({(int32_t)si, t});
      cm_len += (int64_t)g.n_buckets * g.n_tiles;
      nbuck += g.n_buckets;
      gsubs.push_back(g);
    }
    bucket_cm.push_back(cm_len);  // end of the last bucket = total
    HIPCHK(staged(I, I.s_tmp0, gsubs, s));
    HIPCHK(staged(I, I.p_groups, tiles, s));
    HIPCHK(staged(I, I.p_bstart, bucket_cm, s));
    HIPCHK(I.p_cm.ensure((size_t)(cm_len + 1) * 8));
    HIPCHK(I.s_off.ensure((size_t)scan_tmp_elems(cm_len) * 8));
    HIPCHK(I.p_G.ensure((size_t)inst * fmax * 4));
    int32_t fm = fmax;
    HIPCHK(launch_groupby(I.p_asg.as<uint32_t>(), A, &fm, I.s_tmp0.as<GroupSub>(),
                          I.p_groups.as<GroupTile>(), (int32_t)tiles.size(), kGroupTile,
                          I.p_cm.as<int64_t>(), cm_len, I.s_off.as<int64_t>(),
                          I.p_G.as<uint32_t>(), I.p_bstart.as<int64_t>(), nbuck + 1,
                          *std::max_element(ells.begin(), ells.end()), s));
    std::vector<int64_t> bstart((size_t)nbuck + 1);
    HIPCHK(hipMemcpyAsync(bstart.data(), I.p_bstart.p, bstart.size() * 8, hipMemcpyDeviceToHost,
                          s));
    HIPCHK(hipStreamSynchronize(s));
    I.stage.reset();

    // --- plan: merge small buckets, emit leaves, recurse
    std::vector<Sub> next;
    std::vector<Leaf> lv;  // this level's leaves, in output order
    std::vector<const uint32_t *> seg_ptr;
    std::vector<int32_t> seg_len, grp_first;
    std::vector<int64_t> grp_off;
    int64_t gout_total = 0;
    int32_t max_sum = 0;
    std::vector<std::pair<const uint32_t *, int64_t>> recurse_src;
    int64_t next_off = 0;
    const uint32_t *Gp = I.p_G.as<uint32_t>();
    for (size_t si = 0; si < subs.size(); ++si) {
      const Sub &sb = subs[si];
      const int64_t b0 = gsubs[si].bucket_off;
      int64_t gsum = 0;
      int gcnt = 0;
      auto close_group = [&]() {
        if (gcnt == 0) return;
        grp_off.push_back(gout_total);
        gout_total += gsum;
        max_sum = std::max<int32_t>(max_sum, (int32_t)gsum);
        gsum = 0;
        gcnt = 0;
      };
      for (int t = 0; t < ells[si]; ++t) {
        const int64_t st = bstart[(size_t)(b0 + t)];
        const int64_t sz = bstart[(size_t)(b0 + t + 1)] - st;
        if (sz == 0 || sz >= P.c_min) continue;
        if (gcnt > 0 && gsum + sz > P.c_max) close_group();
        if (gcnt == 0) grp_first.push_back((int32_t)seg_ptr.size());
        seg_ptr.push_back(Gp + st);
        seg_len.push_back((int32_t)sz);
        gsum += sz;
        ++gcnt;
      }
      close_group();
      for (int t = 0; t < ells[si]; ++t) {
        const int64_t st = bstart[(size_t)(b0 + t)];
        const int64_t sz = bstart[(size_t)(b0 + t + 1)] - st;
        if (sz == 0 || sz < P.c_min) continue;
        if (sz <= P.c_max) {
          lv.push_back({Gp + st, sz, 0});
        } else if (sz == sb.cnt) {
          const int64_t q = (sz + P.c_max - 1) / P.c_max;
          const int64_t base = sz / q, extra = sz % q;
          int64_t pos = 0;
          for (int64_t c = 0; c < q; ++c) {
            const int64_t len = base + (c < extra ? 1 : 0);
            lv.push_back({Gp + st + pos, len, 0});
            pos += len;
          }
        } else {
          next.push_back({next_off, sz, sub_key(sb.key, t), sb.depth + 1});
          recurse_src.push_back({Gp + st, sz});
          next_off += sz;
        }
      }
    }
    const int n_groups = (int)grp_off.size();
    std::vector<int32_t> grp_size((size_t)n_groups);
    if (n_groups > 0) {
      grp_first.push_back((int32_t)seg_ptr.size());
      HIPCHK(I.p_gout.ensure((size_t)gout_total * 4));
      HIPCHK(staged(I, I.p_seg, seg_ptr, s));
      HIPCHK(staged(I, I.p_seglen, seg_len, s));
      HIPCHK(staged(I, I.p_segfirst, grp_first, s));
      HIPCHK(staged(I, I.p_segoff, grp_off, s));
      HIPCHK(I.p_gsize.ensure((size_t)n_groups * 4));
      HIPCHK(launch_merge_dedup(I.p_seg.as<const uint32_t *>(), I.p_seglen.as<int32_t>(),
                                I.p_segfirst.as<int32_t>(), n_groups, max_sum,
                                I.p_gout.as<uint32_t>(), I.p_segoff.as<int64_t>(),
                                I.p_gsize.as<int32_t>(), s));
      for (int g = 0; g < n_groups; ++g)
        lv.push_back({I.p_gout.as<uint32_t>() + grp_off[(size_t)g], -1, g});
      // the merged sizes
      HIPCHK(hipMemcpyAsync(grp_size.data(), I.p_gsize.p, (size_t)n_groups * 4,
                            hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      I.stage.reset();
    }
    pipnn_status st = emit(lv, grp_size);
    if (st != PIPNN_OK) return st;
    // --- next level: recursing buckets, contiguous
    if (!next.empty()) {
      DevBuf &An = I.p_mem[cur ^ 1];
      HIPCHK(An.ensure((size_t)next_off * 4));
      std::vector<const uint32_t *> src;
      std::vector<int64_t> doff;
      std::vector<int32_t> lens;
      int64_t o = 0;
      for (auto &rs : recurse_src) {
        src.push_back(rs.first);
        doff.push_back(o);
        lens.push_back((int32_t)rs.second);
        o += rs.second;
      }
      HIPCHK(staged(I, I.p_rsrc, src, s));
      HIPCHK(staged(I, I.p_roff, doff, s));
      HIPCHK(staged(I, I.p_rlen, lens, s));
      HIPCHK(launch_copy_segments(I.p_rsrc.as<const uint32_t *>(), I.p_roff.as<int64_t>(),
                                  I.p_rlen.as<int32_t>(), (int32_t)src.size(),
                                  An.as<uint32_t>(), s));
      cur ^= 1;
    }
    subs.swap(next);
  }

  // --- the CSR offsets
  const int64_t n_leaves = (int64_t)offs.size() - 1;
  *h_n_leaves = n_leaves;
  *h_n_members = offs.back();
  if (n_leaves > cap_leaves || offs.back() > cap_members)
    return fail(PIPNN_EOVERFLOW, "partition needs %lld leaves and %lld members",
                (long long)n_leaves, (long long)offs.back());
  if (!d_leaf_offsets || !d_leaf_members) return fail(PIPNN_EINVAL, "NULL output");
  HIPCHK(hipMemcpyAsync(d_leaf_offsets, offs.data(), offs.size() * 8, hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  I.stage.reset();
  I.stats.n_leaves = n_leaves;
  I.stats.n_members = offs.back();
  I.stats.leader_dists = leader_dists;
  I.stats.levels = levels;
  return PIPNN_OK;
  GUARD_END
}

// ---------------------------------------------------------------------
namespace {

struct LeafPlan {
  std::vector<int64_t> offs;  // host copy of the CSR offsets
};

pipnn_status read_offsets(const int64_t *d_off, int64_t n_leaves, hipStream_t s,
                          std::vector<int64_t> &offs) {
  offs.resize((size_t)n_leaves + 1);
  HIPCHK(hipMemcpyAsync(offs.data(), d_off, offs.size() * 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int64_t i = 0; i < n_leaves; ++i) {
    const int64_t sz = offs[(size_t)i + 1] - offs[(size_t)i];
    if (sz < 0) return fail(PIPNN_EINVAL, "leaf offsets are not monotone at leaf %lld", (long long)i);
    if (sz > 65535) return fail(PIPNN_EINVAL, "leaf %lld has %lld > 65535 points", (long long)i,
                                (long long)sz);
  }
  if (offs[0] < 0) return fail(PIPNN_EINVAL, "negative leaf offset");
  return PIPNN_OK;
}

// True when the leaf GEMM's distance already is the value the winners'
// recompute would emit, which is then skipped:
// - the inner product (no norm expansion, hence no cancellation) on an
//   operand that holds the data exactly;
// - the squared L2 distance without rescoring, on integer data whose range
//   makes every form exact in float32 (int_exact), with a float32 operand
//   or a 16-bit copy that holds X exactly: the norm expansion and the
//   direct difference are then the same integer.
static bool gemm_is_direct(const Index &I) {
  if (I.p.metric != PIPNN_METRIC_IP)
    return I.p.metric == PIPNN_METRIC_L2 && !rescoring(I.p) && I.int_exact &&
           (I.p.gemm_prec == PIPNN_PREC_FP32 ||
            (I.op_exact && (I.p.gemm_prec == PIPNN_PREC_BF16 || I.p.gemm_prec == PIPNN_PREC_FP16)));
  return I.p.gemm_prec == PIPNN_PREC_FP32 ||
         (I.p.gemm_prec == PIPNN_PREC_FP16 && I.x_dtype == PIPNN_DTYPE_F16) ||
         (I.p.gemm_prec == PIPNN_PREC_BF16 && I.x_dtype == PIPNN_DTYPE_BF16);
}

// Work list of the pick on leaves [l0, l1) (rows indexed from offs[l0]).
void pick_lists(const Index &I, const std::vector<int64_t> &offs, int64_t l0, int64_t l1,
                std::vector<KnnJob> &jobs, std::vector<KnnItem> &items, int32_t &max_cols,
                int64_t &pairs) {
  const pipnn_params &P = I.p;
  const int ksel = sel_count(P, P.k);
  jobs.clear();
  items.clear();
  max_cols = 0;
  pairs = 0;
  const int64_t base = offs[(size_t)l0];
  for (int64_t l = l0; l < l1; ++l) {
    const int64_t sz = offs[(size_t)l + 1] - offs[(size_t)l];
    if (sz < 2) continue;
    KnnJob J{};
    J.row_off = offs[(size_t)l];
    J.col_off = offs[(size_t)l];
    J.out_off = offs[(size_t)l] - base;
    J.n_rows = (int32_t)sz;
    J.n_cols = (int32_t)sz;
    J.k_sel = ksel;
    J.flags = 1;
    jobs.push_back(J);
    max_cols = std::max<int32_t>(max_cols, (int32_t)sz);
    pairs += sz * sz;
  }
  if (!jobs.empty()) items = plan_items(jobs, 32 * I.leaf_nw);
}

// The same, uploaded into jobs_buf / items_buf.
pipnn_status plan_pick(Index &I, const std::vector<int64_t> &offs, int64_t l0, int64_t l1,
                       DevBuf &jobs_buf, DevBuf &items_buf, int32_t &n_items, int32_t &max_cols,
                       int64_t &pairs, hipStream_t s) {
  std::vector<KnnJob> jobs;
  std::vector<KnnItem> items;
  pick_lists(I, offs, l0, l1, jobs, items, max_cols, pairs);
  n_items = (int32_t)items.size();
  if (jobs.empty()) return PIPNN_OK;
  HIPCHK(upload(jobs_buf, jobs, s));
  HIPCHK(upload(items_buf, items, s));
  return PIPNN_OK;
}

// The pick on a planned work list: clears the picks of `rows` rows, then
// one leaf-kernel launch.
pipnn_status launch_pick(Index &I, const KnnJob *d_jobs, const KnnItem *d_items, int32_t n_items,
                         int32_t max_cols, int64_t rows, const uint32_t *d_members,
                         uint32_t *pick_c, float *pick_d, hipStream_t s, bool local = false) {
  const pipnn_params &P = I.p;
  const int ksel = sel_count(P, P.k);
  HIPCHK(launch_fill_u32(pick_c, kEmptyId, rows * P.k, s));
  HIPCHK(launch_fill_u32(reinterpret_cast<uint32_t *>(pick_d), 0x7F800000u, rows * P.k, s));
  if (n_items == 0) return PIPNN_OK;
  KnnLaunch L{};
  L.idx = &I;
  L.row_base = d_members;
  L.col_base = d_members;
  L.jobs = d_jobs;
  L.items = d_items;
  L.n_items = n_items;
  L.max_cols = max_cols;
  L.ksel = ksel;
  L.k_out = P.k;
  L.out_ids = local ? 0 : 1;
  L.recompute = gemm_is_direct(I) ? 0 : 1;
  L.rescore_k = rescoring(P) ? P.k : 0;
  L.prec = P.gemm_prec;
  L.nw = I.leaf_nw;
  L.persistent = I.leaf_persistent;
  L.quad = I.leaf_quad;
  L.out_col = pick_c;
  L.out_dist = pick_d;
  L.out_matrix = nullptr;
  {
    PhaseTimer t(I, kPhLeafKnn, s);
    HIPCHK(launch_knn(L, s));
  }
  ++I.leaf_launches;
  return PIPNN_OK;
}

// Run the pick on leaves [l0, l1) into picks indexed from offs[l0].
pipnn_status run_pick(Index &I, const std::vector<int64_t> &offs, int64_t l0, int64_t l1,
                      const uint32_t *d_members, uint32_t *pick_c, float *pick_d, hipStream_t s,
                      bool local = false) {
  int32_t n_items = 0, max_cols = 0;
  int64_t pairs = 0;
  pipnn_status st = plan_pick(I, offs, l0, l1, I.s_jobs, I.s_items, n_items, max_cols, pairs, s);
  if (st != PIPNN_OK) return st;
  const int64_t rows = offs[(size_t)l1] - offs[(size_t)l0];
  st = launch_pick(I, I.s_jobs.as<KnnJob>(), I.s_items.as<KnnItem>(), n_items, max_cols, rows,
                   d_members, pick_c, pick_d, s, local);
  I.stats.leaf_pairs += pairs;
  return st;
}

// Scratch of one binning pass: per-point counts (n), bin offsets (n + 1),
// the offsets' scan workspace and the binned records.
struct BinScratch {
  uint32_t *cnt;
  int64_t *off;
  int64_t *tmp0;
  uint64_t *bins;
};

// Bin records by destination and merge them into the reservoirs, with the
// scratch given.
pipnn_status bin_and_merge_in(Index &I, const BinScratch &B, bool from_picks, const uint32_t *a,
                              const uint32_t *b, const float *dist, int64_t count, int32_t k,
                              uint64_t *res, hipStream_t s, bool bidir = true) {
  const int64_t n = I.n;
  {
    PhaseTimer tb(I, kPhBin, s);
    HIPCHK(launch_fill_u32(B.cnt, 0u, n, s));
    if (from_picks)
      HIPCHK(launch_bin_count(a, b, count, k, B.cnt, n, I.flag.as<int32_t>(), s, bidir));
    else
      HIPCHK(launch_rec_count(a, b, count, B.cnt, n, I.flag.as<int32_t>(), s));
    HIPCHK(launch_scan_u32(B.cnt, B.off, n, B.tmp0, s));
    HIPCHK(launch_fill_u32(B.cnt, 0u, n, s));
    if (from_picks)
      HIPCHK(launch_bin_scatter(a, b, dist, count, k, I.sketches.as<float>(), I.m, B.off, B.cnt,
                                B.bins, n, s, bidir));
    else
      HIPCHK(launch_rec_scatter(a, b, dist, count, I.sketches.as<float>(), I.m, B.off, B.cnt,
                                B.bins, n, s));
  }
  {
    PhaseTimer tm(I, kPhMerge, s);
    HIPCHK(launch_hashprune_merge(res, n, I.p.l_max, B.bins, B.off, s));
  }
  return PIPNN_OK;
}

// The same with the index's own scratch.
pipnn_status bin_and_merge(Index &I, bool from_picks, const uint32_t *a, const uint32_t *b,
                           const float *dist, int64_t count, int32_t k, uint64_t *res,
                           hipStream_t s, bool bidir = true) {
  const int64_t n = I.n;
  // every pick yields two records (one when not bidir), every explicit record one
  const int64_t max_rec = from_picks ? (bidir ? 2 : 1) * count * k : count;
  HIPCHK(I.s_cnt.ensure((size_t)n * 4));
  HIPCHK(I.s_off.ensure((size_t)(n + 1) * 8));
  HIPCHK(I.s_tmp0.ensure((size_t)scan_tmp_elems(n) * 8));
  HIPCHK(I.s_bins.ensure((size_t)std::max<int64_t>(max_rec, 1) * 8));
  const BinScratch B{I.s_cnt.as<uint32_t>(), I.s_off.as<int64_t>(), I.s_tmp0.as<int64_t>(),
                     I.s_bins.as<uint64_t>()};
  return bin_and_merge_in(I, B, from_picks, a, b, dist, count, k, res, s, bidir);
}


// All-to-All Prune picks of leaves [l0, l1): the leaf kernel writes each
// leaf's GEMM distance matrix, then one wave per row runs the lazy
// RobustPrune over it. out_ids / out_dist: the batch's rows x k, point ids.
pipnn_status a2a_pick(Index &I, const std::vector<int64_t> &offs, int64_t l0, int64_t l1,
                      const int64_t *d_leaf_off, const uint32_t *d_members, uint32_t *out_ids,
                      float *out_dist, hipStream_t s) {
  const pipnn_params &P = I.p;
  const int64_t rows = offs[(size_t)l1] - offs[(size_t)l0];
  if (rows == 0) return PIPNN_OK;
  int64_t wide = 1;
  for (int64_t l = l0; l < l1; ++l)
    wide = std::max<int64_t>(wide, offs[(size_t)l + 1] - offs[(size_t)l]);
  if (wide > kA2aMaxLeaf)
    return fail(PIPNN_EINVAL, "the all-to-all leaf picker takes leaves of at most %d members",
                kA2aMaxLeaf);
  HIPCHK(I.a2a_mat.ensure((size_t)rows * wide * 4));
  HIPCHK(I.a2a_tmp.ensure((size_t)rows * 8));
  int32_t n_items = 0, max_cols = 0;
  int64_t pairs = 0;
  pipnn_status st = plan_pick(I, offs, l0, l1, I.s_jobs, I.s_items, n_items, max_cols, pairs, s);
  if (st != PIPNN_OK) return st;
  I.stats.leaf_pairs += pairs;
  if (n_items > 0) {
    KnnLaunch L{};
    L.idx = &I;
    L.row_base = d_members;
    L.col_base = d_members;
    L.jobs = I.s_jobs.as<KnnJob>();
    L.items = I.s_items.as<KnnItem>();
    L.n_items = n_items;
    L.max_cols = max_cols;
    L.ksel = 4;  // only the distance matrix is used: the smallest selection
    L.k_out = 1;
    L.out_ids = 0;
    L.recompute = 0;
    L.rescore_k = 0;
    L.prec = P.gemm_prec;
    L.nw = I.leaf_nw;
    L.persistent = I.leaf_persistent;
    L.quad = I.leaf_quad;
    L.out_col = I.a2a_tmp.as<uint32_t>();
    L.out_dist = reinterpret_cast<float *>(I.a2a_tmp.as<uint32_t>() + rows);
    L.out_matrix = I.a2a_mat.as<float>();
    L.matrix_ld = wide;
    PhaseTimer t(I, kPhLeafKnn, s);
    HIPCHK(launch_knn(L, s));
    ++I.leaf_launches;
  }
  PhaseTimer t(I, kPhLeafKnn, s);
  HIPCHK(launch_a2a_prune(I.a2a_mat.as<float>(), wide, d_leaf_off + l0, l1 - l0, offs[(size_t)l0],
                          rows, d_members, I.xf(), I.d, P.metric, gemm_is_direct(I) ? 0 : 1, P.k,
                          P.alpha, out_ids, out_dist, s));
  return PIPNN_OK;
}

// Every leaf's All-to-All Prune picks into out_ids / out_dist (indexed from
// offs[l0]).
pipnn_status a2a_pick_all(Index &I, const std::vector<int64_t> &offs, int64_t l0, int64_t l1,
                          const int64_t *d_leaf_off, const uint32_t *d_members, uint32_t *out_ids,
                          float *out_dist, hipStream_t s) {
  for (auto &b : a2a_batches(offs, l0, l1)) {
    const int64_t o = (offs[(size_t)b.first] - offs[(size_t)l0]) * I.p.k;
    pipnn_status st = a2a_pick(I, offs, b.first, b.second, d_leaf_off, d_members, out_ids + o,
                               out_dist + o, s);
    if (st != PIPNN_OK) return st;
  }
  return PIPNN_OK;
}

// The same for the picks of a batch of leaves written as local column
// indices (leaves of at most kLeafBinMaxRows rows): leaf-local binning.
pipnn_status bin_and_merge_leaves(Index &I, const int64_t *d_leaf_off, int64_t off0,
                                  int64_t n_leaves, const uint32_t *members,
                                  const uint32_t *picks, const float *dist, int64_t rows,
                                  int32_t k, uint64_t *res, hipStream_t s) {
  const int64_t n = I.n;
  const int64_t max_rec = 2 * rows * k;
  HIPCHK(I.s_cnt.ensure((size_t)n * 4));
  HIPCHK(I.s_off.ensure((size_t)(n + 1) * 8));
  HIPCHK(I.s_tmp0.ensure((size_t)scan_tmp_elems(n) * 8));
  HIPCHK(I.s_bins.ensure((size_t)std::max<int64_t>(max_rec, 1) * 8));
  {
    PhaseTimer tb(I, kPhBin, s);
    HIPCHK(launch_fill_u32(I.s_cnt.as<uint32_t>(), 0u, n, s));
    HIPCHK(launch_leaf_bin(false, d_leaf_off, off0, n_leaves, members, picks, dist, k,
                           I.sketches.as<float>(), I.m, nullptr, I.s_cnt.as<uint32_t>(), nullptr,
                           s));
    HIPCHK(launch_scan_u32(I.s_cnt.as<uint32_t>(), I.s_off.as<int64_t>(), n,
                           I.s_tmp0.as<int64_t>(), s));
    HIPCHK(launch_fill_u32(I.s_cnt.as<uint32_t>(), 0u, n, s));
    HIPCHK(launch_leaf_bin(true, d_leaf_off, off0, n_leaves, members, picks, dist, k,
                           I.sketches.as<float>(), I.m, I.s_off.as<int64_t>(),
                           I.s_cnt.as<uint32_t>(), I.s_bins.as<uint64_t>(), s));
  }
  {
    PhaseTimer tm(I, kPhMerge, s);
    HIPCHK(launch_hashprune_merge(res, n, I.p.l_max, I.s_bins.as<uint64_t>(),
                                  I.s_off.as<int64_t>(), s));
  }
  return PIPNN_OK;
}

// Reads the device error flag and the last bin total (one synchronisation).
pipnn_status finish_bins(Index &I, hipStream_t s, const char *what,
                         const int64_t *bin_off = nullptr) {
  int32_t flag = 0;
  int64_t total = 0;
  if (!bin_off) bin_off = I.s_off.as<int64_t>();
  HIPCHK(hipMemcpyAsync(&flag, I.flag.p, 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&total, bin_off + I.n, 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipMemsetAsync(I.flag.p, 0, 4, s));
  I.stats.records += total;
  if (flag) return fail(PIPNN_EDEVICE, "%s: a point id >= n was found on the device", what);
  return PIPNN_OK;
}

__global__ void check_ids_kernel(const uint32_t *ids, int64_t cnt, int64_t n, int32_t *flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt && ids[i] >= n) atomicOr(flag, 1);
}

// (sync) Fails if any of the cnt ids is >= n, before a kernel reads X rows.
pipnn_status check_ids(Index &I, const uint32_t *ids, int64_t cnt, hipStream_t s, const char *what) {
  if (cnt == 0) return PIPNN_OK;
  hipLaunchKernelGGL(check_ids_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, ids,
                     cnt, I.n, I.flag.as<int32_t>());
  HIPCHK(hipGetLastError());
  int32_t flag = 0;
  HIPCHK(hipMemcpyAsync(&flag, I.flag.p, 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (flag) {
    HIPCHK(hipMemsetAsync(I.flag.p, 0, 4, s));
    return fail(PIPNN_EINVAL, "%s: a point id is >= n", what);
  }
  return PIPNN_OK;
}

}  // namespace

// Batches of leaves of at most I.batch_rows rows (a larger leaf is a batch
// of its own), so that the picks and records of a batch fit their scratch.
static std::vector<std::pair<int64_t, int64_t>> leaf_batches(const Index &I,
                                                             const std::vector<int64_t> &offs,
                                                             int64_t n_leaves) {
  const int64_t max_rows = I.batch_rows;
  std::vector<std::pair<int64_t, int64_t>> out;
  int64_t l0 = 0;
  while (l0 < n_leaves) {
    int64_t l1 = l0 + 1;
    while (l1 < n_leaves && offs[(size_t)l1 + 1] - offs[(size_t)l0] <= max_rows) ++l1;
    out.push_back({l0, l1});
    l0 = l1;
  }
  return out;
}

// Device scratch of a build over these batches, allocated up front so that
// a planned build allocates nothing.
static pipnn_status reserve_build(Index &I, const std::vector<int64_t> &offs,
                                  const std::vector<std::pair<int64_t, int64_t>> &batches,
                                  int64_t n_leaves) {
  const int k = I.p.k;
  if (I.ws_mode) {
    // the layout holds the leaves of one partition of the index's points
    const int64_t F = std::max<int64_t>(I.n, members_bound(I.p, I.n));
    const int64_t cnt = offs[(size_t)n_leaves] - offs[0];
    if (cnt > F || n_leaves > F)
      return fail(PIPNN_ENOMEM, "an index on a workspace takes leaves of at most %lld members "
                  "(n times the product of the fanouts); these have %lld in %lld leaves",
                  (long long)F, (long long)cnt, (long long)n_leaves);
  }
  int64_t max_rows = 1;
  for (auto &b : batches)
    max_rows = std::max<int64_t>(max_rows, offs[(size_t)b.second] - offs[(size_t)b.first]);
  const int64_t n = I.n;
  HIPCHK(I.s_picks_c.ensure((size_t)max_rows * k * 4));
  HIPCHK(I.s_picks_d.ensure((size_t)max_rows * k * 4));
  HIPCHK(I.s_cnt.ensure((size_t)n * 4));
  HIPCHK(I.s_off.ensure((size_t)(n + 1) * 8));
  HIPCHK(I.s_tmp0.ensure((size_t)scan_tmp_elems(n) * 8));
  HIPCHK(I.s_bins.ensure((size_t)2 * max_rows * k * 8));
  const int64_t cnt = offs[(size_t)n_leaves] - offs[0];
  const int64_t mx = std::max<int64_t>(cnt, n);
  HIPCHK(I.o_first.ensure((size_t)n * 4));
  HIPCHK(I.o_flag.ensure((size_t)mx * 4));
  HIPCHK(I.o_pos.ensure((size_t)(mx + 1) * 8));
  HIPCHK(I.o_pos2.ensure((size_t)(n + 1) * 8));
  HIPCHK(I.o_tmp.ensure((size_t)scan_tmp_elems(mx) * 8));
  HIPCHK(I.rp_order.ensure((size_t)n * 4));
  HIPCHK(I.lt_off.ensure((size_t)(n_leaves + 1) * 8));
  HIPCHK(I.lt_mem.ensure((size_t)std::max<int64_t>(cnt, 1) * 4));
  return PIPNN_OK;
}

// Keep the leaves of this build for insertion (device copies; the
// representatives are found at the first insertion).
static pipnn_status keep_leaf_table(Index &I, const int64_t *d_off, const uint32_t *d_mem,
                                    const std::vector<int64_t> &offs, int64_t n_leaves,
                                    hipStream_t s) {
  const int64_t cnt = offs[(size_t)n_leaves] - offs[0];
  HIPCHK(launch_rebase_i64(d_off, n_leaves + 1, I.lt_off.as<int64_t>(), s));
  HIPCHK(launch_copy_u32(d_mem + offs[0], cnt, I.lt_mem.as<uint32_t>(), s));
  I.lt_offs.resize((size_t)n_leaves + 1);
  for (int64_t i = 0; i <= n_leaves; ++i) I.lt_offs[(size_t)i] = offs[(size_t)i] - offs[0];
  I.lt_n_leaves = n_leaves;
  I.lt_reps_valid = false;
  return PIPNN_OK;
}

// RobustPrune processing order: points in leaf order.
static pipnn_status leaf_order(Index &I, const uint32_t *d_members, int64_t cnt, hipStream_t s) {
  HIPCHK(launch_leaf_order(d_members, cnt, I.n, I.o_first.as<uint32_t>(),
                           I.o_flag.as<uint32_t>(), I.o_pos.as<int64_t>(),
                           I.o_pos2.as<int64_t>(), I.o_tmp.as<int64_t>(),
                           I.rp_order.as<uint32_t>(), s));
  I.rp_order_valid = true;
  return PIPNN_OK;
}

static bool plan_matches(const Index &I, const int64_t *d_off, const uint32_t *d_mem,
                         int64_t n_leaves) {
  return I.plan.n_leaves == n_leaves && I.plan.d_off == d_off && I.plan.d_mem == d_mem &&
         I.plan.nw == I.leaf_nw;
}

pipnn_status pipnn_plan_leaves(pipnn_index *idx, const int64_t *d_leaf_offsets,
                               const uint32_t *d_leaf_members, int64_t n_leaves,
                               pipnn_stream_t stream) {
  GUARD_BEGIN
  if (idx && reinterpret_cast<Index *>(idx)->p.leaf_picker == PIPNN_PICKER_ALL_TO_ALL)
    return fail(PIPNN_ESTATE, "the all-to-all leaf picker has no planned build");
  if (!idx || !d_leaf_offsets || !d_leaf_members || n_leaves < 1)
    return fail(PIPNN_EINVAL, "invalid argument");
  Index &I = *reinterpret_cast<Index *>(idx);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (stream_capturing(s)) return fail(PIPNN_ESTATE, "plan_leaves cannot run under capture");
  Index::LeafPlan &P = I.plan;
  P.n_leaves = -1;
  pipnn_status st = read_offsets(d_leaf_offsets, n_leaves, s, P.offs);
  if (st != PIPNN_OK) return st;
  st = check_ids(I, d_leaf_members + P.offs[0], P.offs[(size_t)n_leaves] - P.offs[0], s,
                 "plan_leaves");
  if (st != PIPNN_OK) return st;
  auto batches = leaf_batches(I, P.offs, n_leaves);
  st = reserve_build(I, P.offs, batches, n_leaves);
  if (st != PIPNN_OK) return st;
  // every batch's work lists, one after another
  P.batches.assign(batches.size(), Index::PlanBatch{});
  std::vector<KnnJob> all_jobs, jobs;
  std::vector<KnnItem> all_items, items;
  for (size_t i = 0; i < batches.size(); ++i) {
    Index::PlanBatch &B = P.batches[i];
    B.l0 = batches[i].first;
    B.l1 = batches[i].second;
    B.rows = P.offs[(size_t)B.l1] - P.offs[(size_t)B.l0];
    pick_lists(I, P.offs, B.l0, B.l1, jobs, items, B.max_cols, B.pairs);
    B.job_off = (int64_t)all_jobs.size();
    B.item_off = (int64_t)all_items.size();
    B.n_items = (int32_t)items.size();
    all_jobs.insert(all_jobs.end(), jobs.begin(), jobs.end());
    all_items.insert(all_items.end(), items.begin(), items.end());
  }
  HIPCHK(upload(P.jobs, all_jobs, s));
  HIPCHK(upload(P.items, all_items, s));
  HIPCHK(hipStreamSynchronize(s));  // the host work lists may be released now
  P.d_off = d_leaf_offsets;
  P.d_mem = d_leaf_members;
  P.n_leaves = n_leaves;
  P.nw = I.leaf_nw;
  return PIPNN_OK;
  GUARD_END
}

pipnn_status pipnn_build_leaves(pipnn_index *idx, const int64_t *d_leaf_offsets,
                                const uint32_t *d_leaf_members, int64_t n_leaves,
                                uint64_t *d_reservoirs, pipnn_stream_t stream) {
  GUARD_BEGIN
  if (!idx || !d_leaf_offsets || !d_reservoirs || n_leaves < 0)
    return fail(PIPNN_EINVAL, "invalid argument");
  if (n_leaves == 0) return PIPNN_OK;
  if (!d_leaf_members) return fail(PIPNN_EINVAL, "members is NULL");
  Index &I = *reinterpret_cast<Index *>(idx);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int k = I.p.k;
  const bool capturing = stream_capturing(s);
  if (I.p.leaf_picker == PIPNN_PICKER_ALL_TO_ALL) {
    // All-to-All Prune picks of every leaf, then their records (one per
    // admitted candidate) into HashPrune
    if (capturing)
      return fail(PIPNN_ESTATE, "the all-to-all leaf picker has no captured build");
    std::vector<int64_t> offs;
    pipnn_status st = read_offsets(d_leaf_offsets, n_leaves, s, offs);
    if (st != PIPNN_OK) return st;
    I.stats.leaf_pairs = 0;
    I.stats.records = 0;
    const int64_t rows = offs[(size_t)n_leaves] - offs[0];
    st = check_ids(I, d_leaf_members + offs[0], rows, s, "build_leaves");
    if (st != PIPNN_OK) return st;
    const auto batches = leaf_batches(I, offs, n_leaves);
    st = reserve_build(I, offs, batches, n_leaves);
    if (st != PIPNN_OK) return st;
    for (size_t i = 0; i < batches.size(); ++i) {
      const int64_t l0 = batches[i].first, l1 = batches[i].second;
      st = a2a_pick_all(I, offs, l0, l1, d_leaf_offsets, d_leaf_members,
                        I.s_picks_c.as<uint32_t>(), I.s_picks_d.as<float>(), s);
      if (st != PIPNN_OK) return st;
      st = bin_and_merge(I, true, d_leaf_members + offs[(size_t)l0], I.s_picks_c.as<uint32_t>(),
                         I.s_picks_d.as<float>(), offs[(size_t)l1] - offs[(size_t)l0], k,
                         d_reservoirs, s, false);
      if (st != PIPNN_OK) return st;
      if (i + 1 < batches.size()) {
        st = finish_bins(I, s, "build_leaves");
        if (st != PIPNN_OK) return st;
      }
    }
    st = leaf_order(I, d_leaf_members + offs[0], rows, s);
    if (st != PIPNN_OK) return st;
    st = keep_leaf_table(I, d_leaf_offsets, d_leaf_members, offs, n_leaves, s);
    if (st != PIPNN_OK) return st;
    return finish_bins(I, s, "build_leaves");
  }
  const bool planned = plan_matches(I, d_leaf_offsets, d_leaf_members, n_leaves);
  if (capturing && !planned)
    return fail(PIPNN_ESTATE, "build_leaves under stream capture needs pipnn_plan_leaves on the "
                              "same offsets, members and leaf count first");
  pipnn_status st;
  if (planned) {
    // the planned path: device work only
    const Index::LeafPlan &P = I.plan;
    if (!capturing) {
      I.stats.leaf_pairs = 0;
      I.stats.records = 0;
    }
    for (size_t i = 0; i < P.batches.size(); ++i) {
      const Index::PlanBatch &B = P.batches[i];
      const bool local = B.max_cols <= kLeafBinMaxRows;
      st = launch_pick(I, P.jobs.as<KnnJob>() + B.job_off, P.items.as<KnnItem>() + B.item_off,
                       B.n_items, B.max_cols, B.rows, d_leaf_members, I.s_picks_c.as<uint32_t>(),
                       I.s_picks_d.as<float>(), s, local);
      if (st != PIPNN_OK) return st;
      if (!capturing) I.stats.leaf_pairs += B.pairs;
      if (local)
        st = bin_and_merge_leaves(I, d_leaf_offsets + B.l0, P.offs[(size_t)B.l0], B.l1 - B.l0,
                                  d_leaf_members + P.offs[(size_t)B.l0],
                                  I.s_picks_c.as<uint32_t>(), I.s_picks_d.as<float>(), B.rows, k,
                                  d_reservoirs, s);
      else
        st = bin_and_merge(I, true, d_leaf_members + P.offs[(size_t)B.l0],
                           I.s_picks_c.as<uint32_t>(), I.s_picks_d.as<float>(), B.rows, k,
                           d_reservoirs, s);
      if (st != PIPNN_OK) return st;
      if (!capturing && i + 1 < P.batches.size()) {
        st = finish_bins(I, s, "build_leaves");
        if (st != PIPNN_OK) return st;
      }
    }
    st = leaf_order(I, d_leaf_members + P.offs[0], P.offs[(size_t)n_leaves] - P.offs[0], s);
    if (st != PIPNN_OK) return st;
    st = keep_leaf_table(I, d_leaf_offsets, d_leaf_members, P.offs, n_leaves, s);
    if (st != PIPNN_OK) return st;
    return capturing ? PIPNN_OK : finish_bins(I, s, "build_leaves");
  }
  std::vector<int64_t> offs;
  st = read_offsets(d_leaf_offsets, n_leaves, s, offs);
  if (st != PIPNN_OK) return st;
  I.stats.leaf_pairs = 0;
  I.stats.records = 0;
  st = check_ids(I, d_leaf_members + offs[0], offs[(size_t)n_leaves] - offs[0], s, "build_leaves");
  if (st != PIPNN_OK) return st;
  auto batches = leaf_batches(I, offs, n_leaves);
  st = reserve_build(I, offs, batches, n_leaves);
  if (st != PIPNN_OK) return st;
  for (size_t i = 0; i < batches.size(); ++i) {
    const int64_t l0 = batches[i].first, l1 = batches[i].second;
    const int64_t rows = offs[(size_t)l1] - offs[(size_t)l0];
    int64_t biggest = 0;
    for (int64_t l = l0; l < l1; ++l)
      biggest = std::max<int64_t>(biggest, offs[(size_t)l + 1] - offs[(size_t)l]);
    const bool local = biggest <= kLeafBinMaxRows;
    st = run_pick(I, offs, l0, l1, d_leaf_members, I.s_picks_c.as<uint32_t>(),
                  I.s_picks_d.as<float>(), s, local);
    if (st != PIPNN_OK) return st;
    if (local)
      st = bin_and_merge_leaves(I, d_leaf_offsets + l0, offs[(size_t)l0], l1 - l0,
                                d_leaf_members + offs[(size_t)l0], I.s_picks_c.as<uint32_t>(),
                                I.s_picks_d.as<float>(), rows, k, d_reservoirs, s);
    else
      st = bin_and_merge(I, true, d_leaf_members + offs[(size_t)l0], I.s_picks_c.as<uint32_t>(),
                         I.s_picks_d.as<float>(), rows, k, d_reservoirs, s);
    if (st != PIPNN_OK) return st;
    if (i + 1 < batches.size()) {
      st = finish_bins(I, s, "build_leaves");
      if (st != PIPNN_OK) return st;
    }
  }
  st = leaf_order(I, d_leaf_members + offs[0], offs[(size_t)n_leaves] - offs[0], s);
  if (st != PIPNN_OK) return st;
  st = keep_leaf_table(I, d_leaf_offsets, d_leaf_members, offs, n_leaves, s);
  if (st != PIPNN_OK) return st;
  return finish_bins(I, s, "build_leaves");
  GUARD_END
}

// Grow a buffer to `bytes`, keeping its first `keep` bytes.
static hipError_t grow_keep(DevBuf &b, size_t bytes, size_t keep, hipStream_t s) {
  if (b.p && b.cap >= bytes) return hipSuccess;
  DevBuf nb;
  hipError_t e = nb.ensure(bytes);
  if (e != hipSuccess) return e;
  if (b.p && keep) {
    if ((e = hipMemcpyAsync(nb.p, b.p, std::min(keep, b.cap), hipMemcpyDeviceToDevice, s)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess) {
      nb.release();
      return e;
    }
  }
  b.release();
  b = nb;
  return hipSuccess;
}

pipnn_status pipnn_reserve(pipnn_index *idx, int64_t n_cap, const void *d_X,
                           pipnn_stream_t stream) {
  GUARD_BEGIN
  if (!idx) return fail(PIPNN_EINVAL, "NULL index");
  Index &I = *reinterpret_cast<Index *>(idx);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (stream_capturing(s)) return fail(PIPNN_ESTATE, "reserve cannot run under capture");
  if (n_cap >= (int64_t)0xFFFFFFFFll) return fail(PIPNN_EINVAL, "capacity must be < 2^32 - 1");
  if (d_X) {
    // the float32 GEMM operand is X itself unless a padded copy exists, and
    // then it must be 16-byte aligned like the X it replaces
    if (I.x_dtype == PIPNN_DTYPE_F32 && !I.xpad.p && I.ldf != 0 &&
        (reinterpret_cast<uintptr_t>(d_X) & 15u) != 0)
      return fail(PIPNN_EINVAL, "the new X must be 16-byte aligned");
    // the old X may still be read by work on the stream
    HIPCHK(hipStreamSynchronize(s));
    I.X = d_X;
  }
  if (n_cap <= I.cap) return PIPNN_OK;
  if (I.ws_mode)
    return fail(PIPNN_ESTATE, "an index on a caller's workspace holds the %lld points it was "
                "created with", (long long)I.cap);
  const size_t n = (size_t)I.n, c = (size_t)n_cap, d = (size_t)I.d;
  // scratch indexed by point id, sized for the capacity once so that
  // insertions up to it allocate none of it
  HIPCHK(I.s_cnt.ensure(c * 4));
  HIPCHK(I.s_off.ensure((c + 1) * 8));
  HIPCHK(I.s_tmp0.ensure((size_t)scan_tmp_elems(n_cap) * 8));
  HIPCHK(I.i_flag.ensure(c * 4));
  HIPCHK(I.i_pos.ensure((c + 1) * 8));
  HIPCHK(I.i_list.ensure(c * 4));
  HIPCHK(I.o_tmp.ensure((size_t)scan_tmp_elems(n_cap) * 8));
  HIPCHK(grow_keep(I.norms, c * 4, n * 4, s));
  HIPCHK(grow_keep(I.sketches, c * I.m * 4, n * I.m * 4, s));
  if (I.x_dtype != PIPNN_DTYPE_F32) HIPCHK(grow_keep(I.xf32, c * d * 4, n * d * 4, s));
  if (I.xpad.p) HIPCHK(grow_keep(I.xpad, c * I.ldf * 4, n * I.ldf * 4, s));
  if (I.xlow.p) {
    const size_t eb = I.copy_prec == PIPNN_PREC_FP8 ? 1 : 2;
    HIPCHK(grow_keep(I.xlow, c * I.ldo * eb, n * I.ldo * eb, s));
    HIPCHK(grow_keep(I.xscale, c * 4, n * 4, s));
    HIPCHK(grow_keep(I.lnorms, c * 4, n * 4, s));
  }
  if (I.x8.p) {
    HIPCHK(grow_keep(I.x8, c * I.ld8, n * I.ld8, s));
    HIPCHK(grow_keep(I.n8, c * 4, n * 4, s));
  }
  I.cap = n_cap;
  return PIPNN_OK;
  GUARD_END
}

pipnn_status pipnn_insert(pipnn_index *idx, int64_t n_new, const int32_t *d_group,
                          uint64_t *d_reservoirs, uint32_t *d_graph, uint32_t *d_degree,
                          uint64_t epoch, pipnn_stream_t stream) {
  GUARD_BEGIN
  if (!idx || !d_reservoirs || !d_graph || !d_degree || n_new < 0)
    return fail(PIPNN_EINVAL, "invalid argument");
  Index &I = *reinterpret_cast<Index *>(idx);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const uint64_t epoch0 = __atomic_load_n(&I.epoch, __ATOMIC_ACQUIRE);
  if (epoch <= epoch0)
    return fail(PIPNN_EINVAL, "epoch %llu does not follow the index's epoch %llu",
                (unsigned long long)epoch, (unsigned long long)epoch0);
  if (n_new == 0) {
    __atomic_store_n(&I.epoch, epoch, __ATOMIC_RELEASE);
    return PIPNN_OK;
  }
  if (stream_capturing(s)) return fail(PIPNN_ESTATE, "insert cannot run under capture");
  if (I.lt_n_leaves < 1) return fail(PIPNN_ESTATE, "insert needs the leaves of a build first");
  if (I.p.leaf_picker != PIPNN_PICKER_KNN)
    return fail(PIPNN_ESTATE, "insertion picks by the k-NN leaf picker only");
  if (I.n + n_new > I.cap)
    return fail(PIPNN_EOVERFLOW, "insert of %lld points exceeds the reserved capacity %lld",
                (long long)n_new, (long long)I.cap);
  const pipnn_params &P = I.p;
  const int64_t n0 = I.n, n1 = n0 + n_new, d = I.d;
  const int k = P.k;
  const int ksel = sel_count(P, k);
  const int64_t NL = I.lt_n_leaves;
  if (NL > 65535) return fail(PIPNN_EINVAL, "insert routes over at most 65535 leaves");
  if (n_new > 0x7FFFFFFF) return fail(PIPNN_EINVAL, "insert batch too large");

  // 1. the new rows' float32 copy, norms, sketches and GEMM operand (the
  //    count is published atomically for a search running on another thread).
  //    Until the insertion has succeeded, any return restores the count and
  //    the exactness flags that the new rows' checks update, so that a failed
  //    call leaves the index as it was for the next one (the new rows'
  //    buffers and reservoirs are rewritten by it).
  struct Rollback {
    Index &I;
    int64_t n0, int_lo, int_hi;
    bool int_exact, op_exact, i8_ok, done = false;
    ~Rollback() {
      if (done) return;
      __atomic_store_n(&I.n, n0, __ATOMIC_RELEASE);
      I.int_exact = int_exact;
      I.int_lo = int_lo;
      I.int_hi = int_hi;
      I.op_exact = op_exact;
      I.i8_ok = i8_ok;
    }
  } rollback{I, n0, I.int_lo, I.int_hi, I.int_exact, I.op_exact, I.i8_ok};
  __atomic_store_n(&I.n, n1, __ATOMIC_RELEASE);
  I.rp_order_valid = false;  // the leaf order covers the old points only
  if (I.x_dtype != PIPNN_DTYPE_F32) {
    const size_t eb = I.x_dtype == PIPNN_DTYPE_F32 ? 4 : 2;
    HIPCHK(launch_to_f32(reinterpret_cast<const uint8_t *>(I.X) + (size_t)n0 * d * eb, I.x_dtype,
                         I.xf32.as<float>() + n0 * d, n_new * d, s));
  }
  HIPCHK(clear_int_check(I, s));
  HIPCHK(launch_norms_sketches_range(I, n0, n_new, s));
  HIPCHK(read_int_check(I, false, s));
  HIPCHK(launch_pad_range(I, n0, n_new, s));
  // the new rows' int8 rows keep the shift while they stay within its range
  if (I.i8_ok && !(I.int_exact && I.int_lo >= I.lo8 && I.int_hi <= I.lo8 + 255))
    I.i8_ok = false;
  if (I.xlow.p) {
    HIPCHK(clear_op_flag(I, s));
    HIPCHK(launch_quantize_range(I, n0, n_new, s, I.i8_ok));
    HIPCHK(read_op_flag(I, false, s));
  } else if (I.i8_ok) {
    HIPCHK(launch_quantize8_range(I, n0, n_new, s));
  }
  HIPCHK(launch_fill_u64(d_reservoirs + n0 * P.l_max, empty_slot(), n_new * P.l_max, s));

  // 2. route every new point to its f nearest leaves (by the leaf representatives)
  HIPCHK(I.lt_rep.ensure((size_t)NL * 4));
  if (!I.lt_reps_valid) {
    HIPCHK(launch_leaf_reps(I.xf(), I.d, I.lt_off.as<int64_t>(), I.lt_mem.as<uint32_t>(), NL,
                            I.lt_rep.as<uint32_t>(), s));
    I.lt_reps_valid = true;
  }
  const int f = (int)std::min<int64_t>(std::max(1, P.fanout[0]), NL);
  {
    // ids n0 .. n1-1: iota plus n0
    std::vector<KnnJob> jobs(1);
    jobs[0] = KnnJob{};
    jobs[0].n_rows = (int32_t)n_new;
    jobs[0].n_cols = (int32_t)NL;
    jobs[0].k_sel = f;
    std::vector<KnnItem> items = plan_items(jobs, 128);
    HIPCHK(upload(I.s_jobs, jobs, s));
    HIPCHK(upload(I.s_items, items, s));
    std::vector<uint32_t> ids((size_t)n_new);
    for (int64_t i = 0; i < n_new; ++i) ids[(size_t)i] = (uint32_t)(n0 + i);
    HIPCHK(upload(I.i_rows, ids, s));
    HIPCHK(I.i_assign.ensure((size_t)n_new * f * 4));
    KnnLaunch L{};
    L.idx = &I;
    L.row_base = I.i_rows.as<uint32_t>();
    L.col_base = I.lt_rep.as<uint32_t>();
    L.jobs = I.s_jobs.as<KnnJob>();
    L.items = I.s_items.as<KnnItem>();
    L.n_items = (int32_t)items.size();
    L.max_cols = (int32_t)NL;
    L.ksel = f;
    L.k_out = f;
    L.out_ids = 0;
    L.recompute = 0;
    L.rescore_k = 0;
    L.prec = knn_operand_dim(I.d, PIPNN_PREC_FP32) ? PIPNN_PREC_FP32 : P.gemm_prec;
    L.nw = 4;
    L.persistent = 0;
    L.out_col = I.i_assign.as<uint32_t>();
    L.out_dist = nullptr;
    L.out_matrix = nullptr;
    HIPCHK(launch_knn(L, s));
  }
  std::vector<uint32_t> asg((size_t)n_new * f);
  std::vector<int32_t> grp((size_t)n_new, 0);
  HIPCHK(hipMemcpyAsync(asg.data(), I.i_assign.p, asg.size() * 4, hipMemcpyDeviceToHost, s));
  if (d_group)
    HIPCHK(hipMemcpyAsync(grp.data(), d_group, grp.size() * 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));

  // 3. one job per (leaf, group): rows = the group's new points routed to the
  //    leaf; columns = the leaf's members, then those new points
  std::map<std::pair<int64_t, int32_t>, std::vector<uint32_t>> by;
  for (int64_t i = 0; i < n_new; ++i)
    for (int j = 0; j < f; ++j) {
      const uint32_t L = asg[(size_t)i * f + j];
      if (L < (uint32_t)NL) by[{(int64_t)L, grp[(size_t)i]}].push_back((uint32_t)(n0 + i));
    }
  std::vector<KnnJob> jobs;
  std::vector<uint32_t> rows_h, cols_h;
  std::vector<const uint32_t *> seg_src;
  std::vector<int64_t> seg_dst;
  std::vector<int32_t> seg_len;
  for (auto &kv : by) {
    const int64_t L = kv.first.first;
    const auto &pts = kv.second;
    const int64_t mo = I.lt_offs[(size_t)L], ms = I.lt_offs[(size_t)L + 1] - mo;
    if (ms + (int64_t)pts.size() > 65535) return fail(PIPNN_EINVAL, "leaf %lld grows past 65535",
                                                     (long long)L);
    KnnJob J{};
    J.row_off = (int64_t)rows_h.size();
    J.col_off = (int64_t)cols_h.size();
    J.out_off = (int64_t)rows_h.size();
    J.n_rows = (int32_t)pts.size();
    J.n_cols = (int32_t)(ms + (int64_t)pts.size());
    J.k_sel = ksel;
    J.flags = 1;
    J.self_off = (int32_t)ms;
    jobs.push_back(J);
    seg_src.push_back(I.lt_mem.as<uint32_t>() + mo);
    seg_dst.push_back((int64_t)cols_h.size());
    seg_len.push_back((int32_t)ms);
    cols_h.resize(cols_h.size() + (size_t)ms, 0u);
    cols_h.insert(cols_h.end(), pts.begin(), pts.end());
    rows_h.insert(rows_h.end(), pts.begin(), pts.end());
  }
  const int64_t rows = (int64_t)rows_h.size();
  HIPCHK(upload(I.i_rows, rows_h, s));
  HIPCHK(upload(I.i_cols, cols_h, s));
  HIPCHK(upload(I.i_segs, seg_src, s));
  HIPCHK(I.i_tmp.ensure((seg_dst.size() + 1) * 8 + (seg_len.size() + 1) * 4));
  HIPCHK(hipMemcpyAsync(I.i_tmp.p, seg_dst.data(), seg_dst.size() * 8, hipMemcpyHostToDevice, s));
  int32_t *d_len = reinterpret_cast<int32_t *>(I.i_tmp.as<int64_t>() + seg_dst.size() + 1);
  HIPCHK(hipMemcpyAsync(d_len, seg_len.data(), seg_len.size() * 4, hipMemcpyHostToDevice, s));
  HIPCHK(launch_copy_segments(I.i_segs.as<const uint32_t *>(), I.i_tmp.as<int64_t>(), d_len,
                              (int32_t)seg_len.size(), I.i_cols.as<uint32_t>(), s));
  HIPCHK(I.s_picks_c.ensure((size_t)rows * k * 4));
  HIPCHK(I.s_picks_d.ensure((size_t)rows * k * 4));
  {
    std::vector<KnnItem> items = plan_items(jobs, 32 * I.leaf_nw);
    HIPCHK(upload(I.s_jobs, jobs, s));
    HIPCHK(upload(I.s_items, items, s));
    HIPCHK(launch_fill_u32(I.s_picks_c.as<uint32_t>(), kEmptyId, rows * k, s));
    HIPCHK(launch_fill_u32(I.s_picks_d.as<uint32_t>(), 0x7F800000u, rows * k, s));
    KnnLaunch L{};
    L.idx = &I;
    L.row_base = I.i_rows.as<uint32_t>();
    L.col_base = I.i_cols.as<uint32_t>();
    L.jobs = I.s_jobs.as<KnnJob>();
    L.items = I.s_items.as<KnnItem>();
    L.n_items = (int32_t)items.size();
    L.ksel = ksel;
    L.k_out = k;
    L.out_ids = 1;
    L.recompute = gemm_is_direct(I) ? 0 : 1;
    L.rescore_k = rescoring(P) ? k : 0;
    L.prec = P.gemm_prec;
    L.nw = I.leaf_nw;
    L.persistent = 0;
    L.quad = I.leaf_quad;
    L.out_col = I.s_picks_c.as<uint32_t>();
    L.out_dist = I.s_picks_d.as<float>();
    L.out_matrix = nullptr;
    HIPCHK(launch_knn(L, s));
  }
  // 4. both directed records of every pick into HashPrune
  pipnn_status st = bin_and_merge(I, true, I.i_rows.as<uint32_t>(), I.s_picks_c.as<uint32_t>(),
                                  I.s_picks_d.as<float>(), rows, k, d_reservoirs, s);
  if (st != PIPNN_OK) return st;
  // 5. RobustPrune of every point whose reservoir may have changed
  HIPCHK(I.i_flag.ensure((size_t)n1 * 4));
  HIPCHK(I.i_pos.ensure((size_t)(n1 + 1) * 8));
  HIPCHK(I.i_list.ensure((size_t)n1 * 4));
  HIPCHK(I.o_tmp.ensure((size_t)scan_tmp_elems(n1) * 8));
  HIPCHK(launch_fill_u32(I.i_flag.as<uint32_t>(), 0u, n1, s));
  HIPCHK(launch_mark_ids(I.i_rows.as<uint32_t>(), rows, n1, I.i_flag.as<uint32_t>(), s));
  HIPCHK(launch_mark_ids(I.s_picks_c.as<uint32_t>(), rows * k, n1, I.i_flag.as<uint32_t>(), s));
  HIPCHK(launch_scan_u32(I.i_flag.as<uint32_t>(), I.i_pos.as<int64_t>(), n1,
                         I.o_tmp.as<int64_t>(), s));
  HIPCHK(launch_compact_flags(I.i_flag.as<uint32_t>(), I.i_pos.as<int64_t>(), n1,
                              I.i_list.as<uint32_t>(), s));
  int64_t touched = 0;
  HIPCHK(hipMemcpyAsync(&touched, I.i_pos.as<int64_t>() + n1, 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(launch_robustprune(I, d_reservoirs, d_graph, d_degree, I.i_list.as<uint32_t>(), touched,
                            s));
  st = finish_bins(I, s, "insert");
  rollback.done = st == PIPNN_OK;
  if (rollback.done) __atomic_store_n(&I.epoch, epoch, __ATOMIC_RELEASE);
  return st;
  GUARD_END
}

// Whether the index can run leaf picks in this configuration.
static bool leaf_config_ok(const Index &I, int32_t rows_per_item, int32_t persistent,
                           int32_t layout) {
  if (persistent != 0 && persistent != 1) return false;
  if (layout == PIPNN_LAYOUT_QUAD)
    return rows_per_item == 128 && knn_quad_available(I.d, I.p.gemm_prec);
  if (layout != PIPNN_LAYOUT_PAIR || (rows_per_item != 64 && rows_per_item != 128)) return false;
  return knn_pair_available(I.d, I.p.gemm_prec) &&
         knn_nw_available(I.d, I.p.gemm_prec, rows_per_item / 32);
}

pipnn_status pipnn_set_leaf_config(pipnn_index *idx, int32_t rows_per_item, int32_t persistent,
                                   int32_t layout) {
  GUARD_BEGIN
  if (!idx) return fail(PIPNN_EINVAL, "NULL index");
  Index &I = *reinterpret_cast<Index *>(idx);
  if (!leaf_config_ok(I, rows_per_item, persistent, layout))
    return fail(PIPNN_EINVAL, "leaf configuration (%d rows, persistent %d, layout %d) is not built "
                "for this operand", rows_per_item, persistent, layout);
  I.leaf_nw = rows_per_item / 32;
  I.leaf_persistent = persistent;
  I.leaf_quad = layout == PIPNN_LAYOUT_QUAD ? 1 : 0;
  return PIPNN_OK;
  GUARD_END
}

pipnn_status pipnn_autotune(pipnn_index *idx, const int64_t *d_leaf_offsets,
                            const uint32_t *d_leaf_members, int64_t n_leaves,
                            pipnn_tune_result *h_results, int32_t cap_results,
                            int32_t *h_n_results, pipnn_stream_t stream) {
  GUARD_BEGIN
  if (!idx || !d_leaf_offsets || !d_leaf_members || n_leaves < 1)
    return fail(PIPNN_EINVAL, "invalid argument");
  Index &I = *reinterpret_cast<Index *>(idx);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (stream_capturing(s)) return fail(PIPNN_ESTATE, "autotune cannot run under capture");
  std::vector<int64_t> offs;
  pipnn_status st = read_offsets(d_leaf_offsets, n_leaves, s, offs);
  if (st != PIPNN_OK) return st;
  st = check_ids(I, d_leaf_members + offs[0], offs[(size_t)n_leaves] - offs[0], s, "autotune");
  if (st != PIPNN_OK) return st;
  // the first batch of leaves is the sample
  auto batches = leaf_batches(I, offs, n_leaves);
  const int64_t l0 = batches[0].first, l1 = batches[0].second;
  const int64_t rows = offs[(size_t)l1] - offs[(size_t)l0];
  HIPCHK(I.s_picks_c.ensure((size_t)std::max<int64_t>(rows, 1) * I.p.k * 4));
  HIPCHK(I.s_picks_d.ensure((size_t)std::max<int64_t>(rows, 1) * I.p.k * 4));
  std::vector<pipnn_tune_result> res;
  for (int layout : {PIPNN_LAYOUT_PAIR, PIPNN_LAYOUT_QUAD})
    for (int rows : {128, 64})
      for (int pers : {0, 1})
        if (leaf_config_ok(I, rows, pers, layout)) res.push_back({rows, pers, layout, 0.f});
  const int32_t keep_nw = I.leaf_nw, keep_pers = I.leaf_persistent, keep_quad = I.leaf_quad;
  const bool keep_prof = I.profiling;
  I.profiling = false;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  pipnn_status rs = PIPNN_OK;
  for (auto &r : res) {
    I.leaf_nw = r.rows_per_item / 32;
    I.leaf_persistent = r.persistent;
    I.leaf_quad = r.layout == PIPNN_LAYOUT_QUAD ? 1 : 0;
    float best = 1e30f;
    for (int rep = 0; rep < 3 && rs == PIPNN_OK; ++rep) {
      (void)hipEventRecord(e0, s);
      rs = run_pick(I, offs, l0, l1, d_leaf_members + 0, I.s_picks_c.as<uint32_t>(),
                    I.s_picks_d.as<float>(), s);
      (void)hipEventRecord(e1, s);
      if (hipEventSynchronize(e1) != hipSuccess) rs = fail(PIPNN_EDEVICE, "autotune timing failed");
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (rep > 0) best = std::min(best, ms);  // the first run warms up
    }
    r.ms = best;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  I.profiling = keep_prof;
  I.stats.leaf_pairs = 0;
  if (rs != PIPNN_OK) {
    I.leaf_nw = keep_nw;
    I.leaf_persistent = keep_pers;
    I.leaf_quad = keep_quad;
    return rs;
  }
  size_t bi = 0;
  for (size_t i = 1; i < res.size(); ++i)
    if (res[i].ms < res[bi].ms) bi = i;
  I.leaf_nw = res[bi].rows_per_item / 32;
  I.leaf_persistent = res[bi].persistent;
  I.leaf_quad = res[bi].layout == PIPNN_LAYOUT_QUAD ? 1 : 0;
  if (h_n_results) *h_n_results = (int32_t)res.size();
  if (h_results)
    for (size_t i = 0; i < res.size() && (int32_t)i < cap_results; ++i) h_results[i] = res[i];
  return PIPNN_OK;
  GUARD_END
}

pipnn_status pipnn_leaf_pick(pipnn_index *idx, const int64_t *d_leaf_offsets,
                             const uint32_t *d_leaf_members, int64_t n_leaves, uint32_t *d_out_cand,
                             float *d_out_dist, pipnn_stream_t stream) {
  GUARD_BEGIN
  if (!idx || !d_leaf_offsets || !d_out_cand || !d_out_dist || n_leaves < 0)
    return fail(PIPNN_EINVAL, "invalid argument");
  if (n_leaves == 0) return PIPNN_OK;
  Index &I = *reinterpret_cast<Index *>(idx);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  std::vector<int64_t> offs;
  pipnn_status st = read_offsets(d_leaf_offsets, n_leaves, s, offs);
  if (st != PIPNN_OK) return st;
  if (offs[0] != 0) return fail(PIPNN_EINVAL, "offsets[0] must be 0");
  st = check_ids(I, d_leaf_members, offs[(size_t)n_leaves], s, "leaf_pick");
  if (st != PIPNN_OK) return st;
  for (auto &b : leaf_batches(I, offs, n_leaves)) {
    const int64_t o = offs[(size_t)b.first] * I.p.k;
    st = I.p.leaf_picker == PIPNN_PICKER_ALL_TO_ALL
             ? a2a_pick_all(I, offs, b.first, b.second, d_leaf_offsets, d_leaf_members,
                            d_out_cand + o, d_out_dist + o, s)
             : run_pick(I, offs, b.first, b.second, d_leaf_members, d_out_cand + o,
                        d_out_dist + o, s);
    if (st != PIPNN_OK) return st;
  }
  return PIPNN_OK;
  GUARD_END
}

pipnn_status pipnn_knn_block(pipnn_index *idx, const uint32_t *d_row_ids, int64_t n_rows,
                             const uint32_t *d_col_ids, int64_t n_cols, int32_t k,
                             int32_t exclude_diag, uint32_t *d_out_col, float *d_out_dist,
                             float *d_out_matrix, pipnn_stream_t stream) {
  GUARD_BEGIN
  if (!idx || !d_row_ids || !d_col_ids || !d_out_col) return fail(PIPNN_EINVAL, "NULL argument");
  Index &I = *reinterpret_cast<Index *>(idx);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int ksel = sel_count(I.p, k);
  if (k < 1 || ksel > 32) return fail(PIPNN_EINVAL, "k out of range");
  if (n_rows < 1 || n_cols < 1 || n_cols > 65535 || n_rows > 0x7FFFFFFF)
    return fail(PIPNN_EINVAL, "bad block size");
  if (exclude_diag && n_rows != n_cols) return fail(PIPNN_EINVAL, "exclude_diag needs a square block");
  pipnn_status st = check_ids(I, d_row_ids, n_rows, s, "knn_block rows");
  if (st != PIPNN_OK) return st;
  st = check_ids(I, d_col_ids, n_cols, s, "knn_block cols");
  if (st != PIPNN_OK) return st;
  std::vector<KnnJob> jobs(1);
  jobs[0].row_off = 0;
  jobs[0].col_off = 0;
  jobs[0].out_off = 0;
  jobs[0].n_rows = (int32_t)n_rows;
  jobs[0].n_cols = (int32_t)n_cols;
  jobs[0].k_sel = ksel;
  jobs[0].flags = exclude_diag ? 1 : 0;
  std::vector<KnnItem> items = plan_items(jobs, 32 * I.leaf_nw);
  HIPCHK(upload(I.s_jobs, jobs, s));
  HIPCHK(upload(I.s_items, items, s));
  KnnLaunch L{};
  L.idx = &I;
  L.row_base = d_row_ids;
  L.col_base = d_col_ids;
  L.jobs = I.s_jobs.as<KnnJob>();
  L.items = I.s_items.as<KnnItem>();
  L.n_items = (int32_t)items.size();
  L.max_cols = (int32_t)n_cols;
  L.ksel = ksel;
  L.k_out = k;
  L.out_ids = 0;
  L.recompute = gemm_is_direct(I) ? 0 : 1;
  L.rescore_k = rescoring(I.p) ? k : 0;
  L.prec = I.p.gemm_prec;
  L.nw = I.leaf_nw;
  L.persistent = I.leaf_persistent;
  L.quad = I.leaf_quad;
  L.out_col = d_out_col;
  L.out_dist = d_out_dist;
  L.out_matrix = d_out_matrix;
  L.matrix_ld = n_cols;
  HIPCHK(launch_knn(L, s));
  HIPCHK(hipStreamSynchronize(s));
  return PIPNN_OK;
  GUARD_END
}

pipnn_status pipnn_hashprune_insert(pipnn_index *idx, const uint32_t *d_dst,
                                    const uint32_t *d_cand, const float *d_dist,
                                    int64_t n_records, uint64_t *d_reservoirs,
                                    pipnn_stream_t stream) {
  GUARD_BEGIN
  if (!idx || !d_reservoirs || n_records < 0) return fail(PIPNN_EINVAL, "invalid argument");
  if (n_records == 0) return PIPNN_OK;
  if (!d_dst || !d_cand || !d_dist) return fail(PIPNN_EINVAL, "NULL record array");
  Index &I = *reinterpret_cast<Index *>(idx);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  I.stats.records = 0;
  // on a workspace, in chunks that fit the binned-record slice (HashPrune's
  // result does not depend on the order or grouping of its records)
  const int64_t chunk = I.ws_mode ? std::max<int64_t>(1, (int64_t)(I.s_bins.lim / 8)) : n_records;
  for (int64_t r0 = 0; r0 < n_records; r0 += chunk) {
    const int64_t cnt = std::min(chunk, n_records - r0);
    pipnn_status st = bin_and_merge(I, false, d_dst + r0, d_cand + r0, d_dist + r0, cnt, 1,
                                    d_reservoirs, s);
    if (st != PIPNN_OK) return st;
    st = finish_bins(I, s, "hashprune_insert");
    if (st != PIPNN_OK) return st;
  }
  return PIPNN_OK;
  GUARD_END
}

pipnn_status pipnn_hashprune_insert_static(pipnn_index *idx, const uint32_t *d_dst,
                                           const uint32_t *d_cand, const float *d_dist,
                                           int64_t n_records, uint64_t *d_reservoirs,
                                           pipnn_stream_t stream) {
  GUARD_BEGIN
  if (!idx || !d_reservoirs || n_records < 0) return fail(PIPNN_EINVAL, "invalid argument");
  if (n_records == 0) return PIPNN_OK;
  if (!d_dst || !d_cand || !d_dist) return fail(PIPNN_EINVAL, "NULL record array");
  Index &I = *reinterpret_cast<Index *>(idx);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int64_t n = I.n;
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t o_off = 0;
  const size_t o_tmp = o_off + up((size_t)(n + 1) * 8);
  const size_t o_cnt = o_tmp + up((size_t)scan_tmp_elems(n) * 8);
  const size_t o_bins = o_cnt + up((size_t)n * 4);
  const size_t need = o_bins + (size_t)n_records * 8;
  if (need > kStaticScratchBytes)
    return fail(PIPNN_EINVAL,
                "hashprune_insert_static: %lld points and %lld records need %zu bytes of static "
                "scratch; the maximum is %zu",
                (long long)n, (long long)n_records, need, kStaticScratchBytes);
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev != I.device)
    return fail(PIPNN_EINVAL, "hashprune_insert_static: the current device (%d) is not the "
                              "index's (%d)", dev, I.device);
  unsigned char *base = nullptr;
  HIPCHK(static_scratch(dev, &base));
  const BinScratch B{reinterpret_cast<uint32_t *>(base + o_cnt),
                     reinterpret_cast<int64_t *>(base + o_off),
                     reinterpret_cast<int64_t *>(base + o_tmp),
                     reinterpret_cast<uint64_t *>(base + o_bins)};
  I.stats.records = 0;
  pipnn_status st = bin_and_merge_in(I, B, false, d_dst, d_cand, d_dist, n_records, 1,
                                     d_reservoirs, s);
  if (st != PIPNN_OK) return st;
  return finish_bins(I, s, "hashprune_insert_static", B.off);
  GUARD_END
}

pipnn_status pipnn_reservoir_init(uint64_t *d_reservoirs, int64_t n, int32_t l_max,
                                  pipnn_stream_t stream) {
  GUARD_BEGIN
  if (!d_reservoirs || n < 0 || l_max < 1) return fail(PIPNN_EINVAL, "invalid argument");
  HIPCHK(launch_fill_u64(d_reservoirs, empty_slot(), n * (int64_t)l_max,
                         reinterpret_cast<hipStream_t>(stream)));
  return PIPNN_OK;
  GUARD_END
}

pipnn_status pipnn_reservoir_canonical(const pipnn_index *idx, const uint64_t *d_res,
                                       uint64_t *d_out, pipnn_stream_t stream) {
  GUARD_BEGIN
  if (!idx || !d_res || !d_out) return fail(PIPNN_EINVAL, "NULL argument");
  const Index &I = *reinterpret_cast<const Index *>(idx);
  HIPCHK(launch_reservoir_canonical(d_res, d_out, I.n, I.p.l_max,
                                    reinterpret_cast<hipStream_t>(stream)));
  return PIPNN_OK;
  GUARD_END
}

pipnn_status pipnn_robustprune(pipnn_index *idx, const uint64_t *d_reservoirs, uint32_t *d_graph,
                               uint32_t *d_degree, pipnn_stream_t stream) {
  GUARD_BEGIN
  if (!idx || !d_reservoirs || !d_graph || !d_degree) return fail(PIPNN_EINVAL, "NULL argument");
  Index &I = *reinterpret_cast<Index *>(idx);
  PhaseTimer t(I, kPhRobustPrune, reinterpret_cast<hipStream_t>(stream));
  HIPCHK(launch_robustprune(I, d_reservoirs, d_graph, d_degree, nullptr, 0,
                            reinterpret_cast<hipStream_t>(stream)));
  return PIPNN_OK;
  GUARD_END
}

pipnn_status pipnn_start_node(pipnn_index *idx, uint32_t *h_out, pipnn_stream_t stream) {
  GUARD_BEGIN
  if (!idx || !h_out) return fail(PIPNN_EINVAL, "NULL argument");
  Index &I = *reinterpret_cast<Index *>(idx);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int64_t nb = (I.n + 255) / 256;
  HIPCHK(I.s_tmp1.ensure((size_t)(I.d + 2 * nb + 1) * 8 + 8));
  uint32_t *dout = reinterpret_cast<uint32_t *>(I.s_tmp1.as<double>() + I.d + 2 * nb + 1);
  HIPCHK(launch_start_node(I, I.s_tmp1.as<double>(), dout, s));
  HIPCHK(hipMemcpyAsync(h_out, dout, 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return PIPNN_OK;
  GUARD_END
}

pipnn_status pipnn_search(pipnn_index *idx, const uint32_t *d_graph, const void *d_Q, int64_t nq,
                          int32_t q_dtype, int32_t k, int32_t L, uint32_t start,
                          uint32_t *d_out_ids, float *d_out_dist, uint32_t *d_out_cmps,
                          pipnn_stream_t stream) {
  GUARD_BEGIN
  if (!idx || !d_graph || !d_out_ids || (!d_Q && nq > 0) || nq < 0)
    return fail(PIPNN_EINVAL, "invalid argument");
  Index &I = *reinterpret_cast<Index *>(idx);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (k < 1 || k > L || L > 1024) return fail(PIPNN_EINVAL, "need 1 <= k <= L <= 1024");
  // one reading of the point count: an insertion on another thread may grow it
  const int64_t n = __atomic_load_n(&I.n, __ATOMIC_ACQUIRE);
  if ((int64_t)start >= n) return fail(PIPNN_EINVAL, "start >= n");
  if (q_dtype != PIPNN_DTYPE_F32 && q_dtype != PIPNN_DTYPE_F16 && q_dtype != PIPNN_DTYPE_BF16)
    return fail(PIPNN_EINVAL, "unknown q_dtype");
  if (nq == 0) return PIPNN_OK;
  // batches of queries whose seen bitmaps (n bits each) fit the budget; a
  // 16-bit batch is widened to float32 first
  const int64_t words = (n + 31) / 32;
  const int64_t batch = std::min<int64_t>(nq, query_batch(n));
  HIPCHK(I.q_seen.ensure((size_t)batch * words * 4));
  if (q_dtype != PIPNN_DTYPE_F32) HIPCHK(I.q_conv.ensure((size_t)batch * I.d * 4));
  const size_t qrow = (size_t)I.d * (q_dtype == PIPNN_DTYPE_F32 ? 4 : 2);
  for (int64_t q0 = 0; q0 < nq; q0 += batch) {
    const int64_t nb = std::min(batch, nq - q0);
    const void *qb = static_cast<const char *>(d_Q) + (size_t)q0 * qrow;
    const float *Q = reinterpret_cast<const float *>(qb);
    if (q_dtype != PIPNN_DTYPE_F32) {
      HIPCHK(launch_to_f32(qb, q_dtype, I.q_conv.as<float>(), nb * (int64_t)I.d, s));
      Q = I.q_conv.as<float>();
    }
    HIPCHK(hipMemsetAsync(I.q_seen.p, 0, (size_t)nb * words * 4, s));
    HIPCHK(launch_search(I, n, d_graph, Q, nb, k, L, start, d_out_ids + q0 * k,
                         d_out_dist ? d_out_dist + q0 * k : nullptr,
                         d_out_cmps ? d_out_cmps + q0 : nullptr, I.q_seen.as<uint32_t>(), words,
                         s));
  }
  return PIPNN_OK;
  GUARD_END
}

pipnn_status pipnn_knn_graph(pipnn_index *idx, const uint32_t *d_graph, int32_t k, int32_t L,
                             uint32_t start, uint32_t *d_out_ids, float *d_out_dist,
                             pipnn_stream_t stream) {
  GUARD_BEGIN
  if (!idx || !d_graph || !d_out_ids) return fail(PIPNN_EINVAL, "NULL argument");
  Index &I = *reinterpret_cast<Index *>(idx);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (k < 1 || k + 1 > L || L > 1024) return fail(PIPNN_EINVAL, "need 1 <= k < L <= 1024");
  const int64_t n = I.n;
  if ((int64_t)start >= n) return fail(PIPNN_EINVAL, "start >= n");
  const int64_t words = (n + 31) / 32;
  const int32_t k1 = k + 1;
  int64_t chunk = std::min<int64_t>(n, query_batch(n));
  // on a workspace the result slices hold a chunk of k + 1 <= 65 results
  if (I.ws_mode) chunk = std::max<int64_t>(1, std::min<int64_t>(chunk, I.g_ids.lim / (k1 * 4)));
  HIPCHK(I.q_seen.ensure((size_t)chunk * words * 4));
  HIPCHK(I.g_ids.ensure((size_t)chunk * k1 * 4));
  HIPCHK(I.g_dist.ensure((size_t)chunk * k1 * 4));
  for (int64_t q0 = 0; q0 < n; q0 += chunk) {
    const int64_t nb = std::min(chunk, n - q0);
    HIPCHK(hipMemsetAsync(I.q_seen.p, 0, (size_t)nb * words * 4, s));
    HIPCHK(launch_search(I, n, d_graph, I.xf() + q0 * I.d, nb, k1, L, start,
                         I.g_ids.as<uint32_t>(), I.g_dist.as<float>(), nullptr,
                         I.q_seen.as<uint32_t>(), words, s));
    HIPCHK(launch_drop_self(I.g_ids.as<uint32_t>(), I.g_dist.as<float>(), nb, k1, q0, d_out_ids,
                            d_out_dist, s));
  }
  return PIPNN_OK;
  GUARD_END
}

pipnn_status pipnn_prepare(pipnn_index *idx, pipnn_stream_t stream) {
  GUARD_BEGIN
  if (!idx) return fail(PIPNN_EINVAL, "NULL index");
  Index &I = *reinterpret_cast<Index *>(idx);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  PhaseTimer t(I, kPhPrepare, s);
  if (I.x_dtype != PIPNN_DTYPE_F32)
    HIPCHK(launch_to_f32(I.X, I.x_dtype, I.xf32.as<float>(), I.n * (int64_t)I.d, s));
  HIPCHK(clear_int_check(I, s));
  HIPCHK(launch_norms_sketches(I, s));
  // outside capture the integer check is taken again (as the operand's
  // exactness below); a captured prepare keeps the last one
  if (!stream_capturing(s)) HIPCHK(read_int_check(I, true, s));
  HIPCHK(launch_pad_range(I, 0, I.n, s));
  if (I.p.gemm_prec != PIPNN_PREC_FP32) {
    HIPCHK(clear_op_flag(I, s));
    HIPCHK(launch_quantize(I, s));
    // outside capture the operand's exactness is taken again; a captured
    // prepare keeps the one found by the last uncaptured encode
    if (!stream_capturing(s)) HIPCHK(read_op_flag(I, true, s));
    HIPCHK(refresh_rows8(I, s));
  } else {
    HIPCHK(refresh_fp32_copy(I, s));
  }
  return PIPNN_OK;
  GUARD_END
}

pipnn_status pipnn_set_profiling(pipnn_index *idx, int32_t on) {
  GUARD_BEGIN
  if (!idx) return fail(PIPNN_EINVAL, "NULL index");
  Index &I = *reinterpret_cast<Index *>(idx);
  flush_events(I);
  for (double &v : I.phase_ms) v = 0.0;
  I.leaf_launches = 0;
  I.profiling = on != 0;
  return PIPNN_OK;
  GUARD_END
}

pipnn_status pipnn_get_stats(pipnn_index *idx, pipnn_stats *h_out) {
  GUARD_BEGIN
  if (!idx || !h_out) return fail(PIPNN_EINVAL, "NULL argument");
  Index &I = *reinterpret_cast<Index *>(idx);
  flush_events(I);
  pipnn_stats st = I.stats;
  st.leaf_knn_launches = I.leaf_launches;
  st.operand_exact = I.op_exact ? 1 : 0;
  st.data_int_exact = I.int_exact ? 1 : 0;
  st.rp_row_bits = rp_row_bits(I);
  st.ms_prepare = I.phase_ms[kPhPrepare];
  st.ms_partition = I.phase_ms[kPhPartition];
  st.ms_leaf_knn = I.phase_ms[kPhLeafKnn];
  st.ms_bin = I.phase_ms[kPhBin];
  st.ms_merge = I.phase_ms[kPhMerge];
  st.ms_robustprune = I.phase_ms[kPhRobustPrune];
  st.epoch = __atomic_load_n(&I.epoch, __ATOMIC_ACQUIRE);
  st.n_points = __atomic_load_n(&I.n, __ATOMIC_ACQUIRE);
  st.workspace_bytes = (int64_t)I.ws_bytes;
  st.batch_rows = I.batch_rows;
  *h_out = st;
  return PIPNN_OK;
  GUARD_END
}

pipnn_status pipnn_get_sketches(const pipnn_index *idx, float *d_out, pipnn_stream_t stream) {
  GUARD_BEGIN
  if (!idx || !d_out) return fail(PIPNN_EINVAL, "NULL argument");
  const Index &I = *reinterpret_cast<const Index *>(idx);
  HIPCHK(hipMemcpyAsync(d_out, I.sketches.p, (size_t)I.n * I.m * 4, hipMemcpyDeviceToDevice,
                        reinterpret_cast<hipStream_t>(stream)));
  return PIPNN_OK;
  GUARD_END
}

pipnn_status pipnn_get_operand(const pipnn_index *idx, void *d_codes, float *d_scale,
                               float *d_norms, pipnn_stream_t stream) {
  GUARD_BEGIN
  if (!idx) return fail(PIPNN_EINVAL, "NULL index");
  const Index &I = *reinterpret_cast<const Index *>(idx);
  if (I.p.gemm_prec == PIPNN_PREC_FP32)
    return fail(PIPNN_ESTATE, "the index has no reduced-precision operand");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const size_t eb = I.p.gemm_prec == PIPNN_PREC_FP8 ? 1 : 2;
  if (d_codes)
    HIPCHK(hipMemcpy2DAsync(d_codes, (size_t)I.d * eb, I.xlow.p, (size_t)I.ldo * eb,
                            (size_t)I.d * eb, (size_t)I.n, hipMemcpyDeviceToDevice, s));
  if (d_scale) {
    if (I.p.gemm_prec == PIPNN_PREC_FP8)
      HIPCHK(hipMemcpyAsync(d_scale, I.xscale.p, (size_t)I.n * 4, hipMemcpyDeviceToDevice, s));
    else
      HIPCHK(launch_fill_u32(reinterpret_cast<uint32_t *>(d_scale), 0x3F800000u, I.n, s));
  }
  if (d_norms)
    HIPCHK(hipMemcpyAsync(d_norms, I.lnorms.p, (size_t)I.n * 4, hipMemcpyDeviceToDevice, s));
  return PIPNN_OK;
  GUARD_END
}

}  // extern "C"

// C ABI of the solver: argument validation, device tables, work-buffer
// layout and the host-side step drivers.  Every step of the method runs in
// the kernels of kernels.hip; this file only orders launches on the caller's
// stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "engine.hpp"

using namespace gpe;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string t_err;

static gpe_status fail(gpe_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  t_err = buf;
  return st;
}

static gpe_status hip_fail(hipError_t e, const char* what) {
  return fail(GPE_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr)                                   \
  do {                                                  \
    hipError_t _e = (expr);                             \
    if (_e != hipSuccess) return hip_fail(_e, #expr);   \
  } while (0)

struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (dev >= 0 && dev != prev) ok = (hipSetDevice(dev) == hipSuccess);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

// ---------------------------------------------------------------------------
// per-kernel timing
// ---------------------------------------------------------------------------
namespace {
struct TimingState {
  bool enabled = false;
  int64_t launches[FAM_COUNT] = {0};
  double ms[FAM_COUNT] = {0};
  struct Pending { int fam; hipEvent_t a, b; };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  hipEvent_t open_a = nullptr;
  int open_fam = -1;
};
TimingState g_tim;

hipEvent_t pool_get() {
  if (!g_tim.pool.empty()) {
    hipEvent_t e = g_tim.pool.back();
    g_tim.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void resolve_pending(size_t keep) {
  while (g_tim.pending.size() > keep) {
    TimingState::Pending p = g_tim.pending.front();
    g_tim.pending.erase(g_tim.pending.begin());
    float ms = 0.f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      g_tim.ms[p.fam] += ms;
      g_tim.launches[p.fam] += 1;
    }
    g_tim.pool.push_back(p.a);
    g_tim.pool.push_back(p.b);
  }
}

bool capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess) return false;
  return st != hipStreamCaptureStatusNone;
}
}  // namespace

namespace gpe {
void timing_before(int fam, hipStream_t s) {
  if (!g_tim.enabled || capturing(s)) return;
  hipEvent_t a = pool_get();
  if (!a) return;
  if (hipEventRecord(a, s) != hipSuccess) {
    g_tim.pool.push_back(a);
    return;
  }
  g_tim.open_a = a;
  g_tim.open_fam = fam;
}
void timing_after(int fam, hipStream_t s) {
  if (!g_tim.enabled || g_tim.open_a == nullptr || g_tim.open_fam != fam) return;
  hipEvent_t b = pool_get();
  if (!b || hipEventRecord(b, s) != hipSuccess) {
    g_tim.pool.push_back(g_tim.open_a);
    if (b) g_tim.pool.push_back(b);
    g_tim.open_a = nullptr;
    return;
  }
  g_tim.pending.push_back({fam, g_tim.open_a, b});
  g_tim.open_a = nullptr;
  if (g_tim.pending.size() > 16384) resolve_pending(8192);
}
}  // namespace gpe

// ---------------------------------------------------------------------------
// problem: one or more instances in one concatenated compact layout
// ---------------------------------------------------------------------------
namespace {

template <typename T>
hipError_t dalloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  return hipMalloc((void**)p, count * sizeof(T));
}

struct ChunkSet {
  int capacity = 0;
  int n_chunks = 0;
  int max_seg = 1;
  Chunk* d_chunks = nullptr;
  GroupSegs* d_groups = nullptr;       // capacity / 64 per chunk
  int32_t* d_order = nullptr;          // workgroup -> chunk for order mode 4 (built on first use)
  std::vector<int> inst_begin, inst_count;
  std::vector<int32_t> site_begin;     // host copy of each chunk's first site
};

struct Problem {
  int device = -1;
  int n_inst = 0;
  int64_t total = 0;
  int64_t n_segs = 0;
  std::vector<int64_t> inst_site;      // n_inst + 1
  std::vector<int64_t> inst_seg;       // n_inst + 1
  std::vector<double> inst_h;          // 3 per instance
  std::vector<SegHead> heads;          // host copy (n_segs + 1)
  std::vector<int64_t> plane_begin;    // first compact site of every non-empty x-plane of every instance
  // 19- and 27-point stencil tables (single grids only, built by enable_hoc)
  int stencil = 7;
  std::vector<SegHead> hoc_heads, c27_heads;   // host copies (segments + 1)
  SegHead* d_hoc_heads = nullptr;
  SegHoc* d_hoc_nbs = nullptr;
  SegHead* d_c27_heads = nullptr;
  SegC27* d_c27_nbs = nullptr;
  SegHead* d_heads = nullptr;
  SegNb* d_nbs = nullptr;
  std::map<int, ChunkSet> chunksets;
  InstParams* d_inst = nullptr;
  InstOut* d_out = nullptr;
  int64_t* d_step = nullptr;
  double* d_partials = nullptr;
  double* d_knot_acc = nullptr;
  double* d_grads = nullptr;
  int64_t max_chunks = 0;
  InstParams* h_inst = nullptr;        // pinned staging
  hipEvent_t upload_done = nullptr;
  // End of the last call's work on the handle.  The instance table, results,
  // partial sums and step counter are shared by every call, so a call on
  // another stream first waits for it (calls on one stream are ordered anyway).
  hipEvent_t last_done = nullptr;
  hipStream_t last_stream = nullptr;
  bool has_last = false;
  int config = 0;
  // captured forward-step graphs, keyed by buffer pointers
  struct GraphKey {
    const void *psi, *field, *work;
    int dtype, config, scheme, integrator, stencil;
    bool operator<(const GraphKey& o) const {
      return std::tie(psi, field, work, dtype, config, scheme, integrator, stencil) <
             std::tie(o.psi, o.field, o.work, o.dtype, o.config, o.scheme, o.integrator, o.stencil);
    }
  };
  std::map<GraphKey, hipGraphExec_t> graphs;

  ~Problem() { release(); }
  void release() {
    if (device < 0) return;
    DeviceGuard g(device);
    (void)hipDeviceSynchronize();     // launches and graphs in flight use these tables
    for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
    graphs.clear();
    for (auto& kv : chunksets) {
      (void)hipFree(kv.second.d_chunks);
      (void)hipFree(kv.second.d_groups);
      (void)hipFree(kv.second.d_order);
    }
    chunksets.clear();
    (void)hipFree(d_heads);
    (void)hipFree(d_nbs);
    (void)hipFree(d_hoc_heads);
    (void)hipFree(d_hoc_nbs);
    (void)hipFree(d_c27_heads);
    (void)hipFree(d_c27_nbs);
    d_hoc_heads = nullptr;
    d_hoc_nbs = nullptr;
    d_c27_heads = nullptr;
    d_c27_nbs = nullptr;
    (void)hipFree(d_inst);
    (void)hipFree(d_out);
    (void)hipFree(d_step);
    (void)hipFree(d_partials);
    (void)hipFree(d_knot_acc);
    (void)hipFree(d_grads);
    if (h_inst) (void)hipHostFree(h_inst);
    if (upload_done) (void)hipEventDestroy(upload_done);
    if (last_done) (void)hipEventDestroy(last_done);
    last_done = nullptr;
    has_last = false;
    d_heads = nullptr;
    d_nbs = nullptr;
    d_inst = nullptr;
    d_out = nullptr;
    d_step = nullptr;
    d_partials = d_knot_acc = d_grads = nullptr;
    h_inst = nullptr;
    upload_done = nullptr;
    device = -1;
  }

  // Build from instance layouts (concatenated in order).
  gpe_status build(int dev, const std::vector<const Layout*>& lays) {
    device = dev;
    n_inst = (int)lays.size();
    inst_site.assign(n_inst + 1, 0);
    inst_seg.assign(n_inst + 1, 0);
    inst_h.assign(3 * n_inst, 0.0);
    for (int i = 0; i < n_inst; ++i) {
      inst_site[i + 1] = inst_site[i] + lays[i]->n_active;
      inst_seg[i + 1] = inst_seg[i] + lays[i]->n_segments();
      for (int d = 0; d < 3; ++d) inst_h[3 * i + d] = lays[i]->h[d];
    }
    total = inst_site[n_inst];
    n_segs = inst_seg[n_inst];
    if (total > (int64_t)INT32_MAX - 1) return fail(GPE_ERR_ARG, "more than 2^31-2 active sites in total");
    heads.resize(n_segs + 1);
    std::vector<SegNb> nbs(n_segs);
    for (int i = 0; i < n_inst; ++i) {
      const Layout& L = *lays[i];
      for (int64_t q = 0; q < L.n_segments(); ++q) {
        SegHead h = L.heads[q];
        h.start += (int32_t)inst_site[i];
        heads[inst_seg[i] + q] = h;
        nbs[inst_seg[i] + q] = L.nbs[q];
      }
    }
    heads[n_segs] = {(int32_t)total, 0};
    plane_begin.clear();
    for (int i = 0; i < n_inst; ++i) {
      const Layout& L = *lays[i];
      for (int64_t r = 0; r < L.n_runs(); ++r)
        if (r == 0 || L.run_i[r] != L.run_i[r - 1]) plane_begin.push_back(inst_site[i] + L.run_start[r]);
    }
    DeviceGuard g(device);
    if (!g.ok) return fail(GPE_ERR_DEVICE, "hipSetDevice(%d) failed", device);
    // chunks of >= 256 sites each, plus at most one extra chunk per
    // MAX_CHUNK_SEGS segments where a fragmented mask cuts chunks short
    max_chunks = 0;
    for (int i = 0; i < n_inst; ++i)
      max_chunks += (lays[i]->n_active + 255) / 256 + lays[i]->n_segments() / MAX_CHUNK_SEGS + 1;
    if (dalloc(&d_heads, n_segs + 1) != hipSuccess || dalloc(&d_nbs, n_segs) != hipSuccess ||
        dalloc(&d_inst, n_inst) != hipSuccess || dalloc(&d_out, n_inst) != hipSuccess ||
        dalloc(&d_step, 1) != hipSuccess || dalloc(&d_partials, max_chunks * NPART) != hipSuccess ||
        dalloc(&d_knot_acc, max_chunks * GPE_MAX_KNOTS) != hipSuccess ||
        dalloc(&d_grads, (size_t)n_inst * GPE_MAX_KNOTS) != hipSuccess) {
      release();
      return fail(GPE_ERR_ALLOC, "device allocation of grid tables failed");
    }
    if (hipHostMalloc((void**)&h_inst, sizeof(InstParams) * n_inst) != hipSuccess) {
      h_inst = nullptr;
      release();
      return fail(GPE_ERR_ALLOC, "pinned host allocation failed");
    }
    if (hipEventCreateWithFlags(&upload_done, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&last_done, hipEventDisableTiming) != hipSuccess) {
      release();
      return fail(GPE_ERR_DEVICE, "hipEventCreate failed");
    }
    hipError_t e = hipMemcpy(d_heads, heads.data(), sizeof(SegHead) * (n_segs + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess && n_segs > 0)
      e = hipMemcpy(d_nbs, nbs.data(), sizeof(SegNb) * n_segs, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(d_out, 0, sizeof(InstOut) * n_inst);
    if (e == hipSuccess) e = hipMemset(d_step, 0, sizeof(int64_t));
    if (e != hipSuccess) {
      gpe_status st = hip_fail(e, "upload of grid tables");
      release();
      return st;
    }
    return GPE_OK;
  }

  // Upload the 19-point segment tables of a single grid's layout (built on
  // the host on first use) and make sure the partial-sum scratch covers the
  // larger chunk count.
  template <typename Desc>
  gpe_status upload_taps(const std::vector<SegHead>& hh, const std::vector<Desc>& nb, SegHead** dh, Desc** dn) {
    const int64_t nh = (int64_t)nb.size();
    DeviceGuard g(device);
    if (dalloc(dh, nh + 1) != hipSuccess || dalloc(dn, nh) != hipSuccess) {
      (void)hipFree(*dh);
      (void)hipFree(*dn);
      *dh = nullptr;
      *dn = nullptr;
      return fail(GPE_ERR_ALLOC, "stencil segment table allocation failed");
    }
    hipError_t e = hipMemcpy(*dh, hh.data(), sizeof(SegHead) * (nh + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(*dn, nb.data(), sizeof(Desc) * nh, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(*dh);
      (void)hipFree(*dn);
      *dh = nullptr;
      *dn = nullptr;
      return hip_fail(e, "stencil segment table upload");
    }
    return GPE_OK;
  }

  gpe_status enable_hoc(Layout& lay, int points) {
    if (n_inst != 1) return fail(GPE_ERR_STATE, "the 19- and 27-point stencils are available for single grids only");
    int64_t nh = 0;
    if (points == 19) {
      if (d_hoc_heads) return GPE_OK;
      build_hoc_segments(lay);
      hoc_heads = lay.hoc_heads;
      nh = (int64_t)lay.hoc_nbs.size();
      gpe_status st = upload_taps(hoc_heads, lay.hoc_nbs, &d_hoc_heads, &d_hoc_nbs);
      if (st != GPE_OK) return st;
    } else {
      if (d_c27_heads) return GPE_OK;
      build_c27_segments(lay);
      c27_heads = lay.c27_heads;
      nh = (int64_t)lay.c27_nbs.size();
      gpe_status st = upload_taps(c27_heads, lay.c27_nbs, &d_c27_heads, &d_c27_nbs);
      if (st != GPE_OK) return st;
    }
    DeviceGuard g(device);
    const int64_t need = (lay.n_active + 255) / 256 + nh / MAX_CHUNK_SEGS + 1;
    if (need > max_chunks) {
      // the graphs and launches in flight hold the old scratch
      if (hipDeviceSynchronize() != hipSuccess) return fail(GPE_ERR_DEVICE, "hipDeviceSynchronize failed");
      for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
      graphs.clear();
      (void)hipFree(d_partials);
      (void)hipFree(d_knot_acc);
      d_partials = d_knot_acc = nullptr;
      max_chunks = need;
      if (dalloc(&d_partials, max_chunks * NPART) != hipSuccess ||
          dalloc(&d_knot_acc, max_chunks * GPE_MAX_KNOTS) != hipSuccess)
        return fail(GPE_ERR_ALLOC, "partial-sum scratch allocation failed");
    }
    return GPE_OK;
  }

  // chunk table for a chunk capacity and stencil (built on first use)
  gpe_status chunks_for(int capacity, ChunkSet** out, int points = 7, bool build = true) {
    const int key = capacity * 4 + (points == 19 ? 1 : (points == 27 ? 2 : 0));
    auto it = chunksets.find(key);
    if (it != chunksets.end()) {
      *out = &it->second;
      return GPE_OK;
    }
    if (!build) return fail(GPE_ERR_STATE, "internal: the chunk table of the grid's launch variant is not built");
    const std::vector<SegHead>& heads = points == 19 ? hoc_heads : (points == 27 ? c27_heads : this->heads);
    ChunkSet cs;
    cs.capacity = capacity;
    std::vector<Chunk> tab;
    cs.inst_begin.resize(n_inst);
    cs.inst_count.resize(n_inst);
    for (int i = 0; i < n_inst; ++i) {
      cs.inst_begin[i] = (int)tab.size();
      int64_t seg = inst_seg[i];
      for (int64_t b = inst_site[i]; b < inst_site[i + 1];) {
        int64_t e = std::min<int64_t>(b + capacity, inst_site[i + 1]);
        while (heads[seg + 1].start <= b) ++seg;
        int64_t last = seg;
        while (heads[last + 1].start <= e - 1) ++last;
        if (last - seg + 1 > MAX_CHUNK_SEGS) {
          // end the chunk where its (MAX_CHUNK_SEGS + 1)-th segment begins
          last = seg + MAX_CHUNK_SEGS - 1;
          e = heads[last + 1].start;
        }
        Chunk c;
        c.site_begin = (int32_t)b;
        c.count = (int32_t)(e - b);
        c.seg_begin = (int32_t)seg;
        c.seg_count = (int32_t)(last - seg + 1);
        c.inst = i;
        c.pad[0] = c.pad[1] = c.pad[2] = 0;
        cs.max_seg = std::max(cs.max_seg, c.seg_count);
        tab.push_back(c);
        cs.site_begin.push_back(c.site_begin);
        b = e;
      }
      cs.inst_count[i] = (int)tab.size() - cs.inst_begin[i];
    }
    cs.n_chunks = (int)tab.size();
    if ((int64_t)cs.n_chunks > max_chunks) return fail(GPE_ERR_STATE, "internal: chunk count exceeds scratch");
    if (capacity % 64 != 0) return fail(GPE_ERR_STATE, "internal: chunk capacity is not a multiple of 64");
    // segment starts of every 64-site group of every chunk
    const int G = capacity / 64;
    std::vector<GroupSegs> groups((size_t)cs.n_chunks * G);
    for (size_t c = 0; c < tab.size(); ++c) {
      const Chunk& ch = tab[c];
      GroupSegs* gs = &groups[c * G];
      for (int q = 0; q < G; ++q) gs[q] = GroupSegs{0ull, ch.seg_count - 1, 0};
      int k = 0;   // chunk-relative segment holding the current group's first site
      for (int q = 0; q < G && 64 * q < ch.count; ++q) {
        const int64_t b = (int64_t)ch.site_begin + 64 * q;
        const int64_t e = std::min<int64_t>(b + 64, (int64_t)ch.site_begin + ch.count);
        while (k + 1 < ch.seg_count && heads[ch.seg_begin + k + 1].start <= b) ++k;
        gs[q].first = k;
        for (int j = k; j < ch.seg_count; ++j) {
          const int64_t st = heads[ch.seg_begin + j].start;
          if (st >= e) break;
          if (st >= b) gs[q].starts |= 1ull << (st - b);
        }
      }
    }
    DeviceGuard g(device);
    if (dalloc(&cs.d_chunks, tab.size()) != hipSuccess) return fail(GPE_ERR_ALLOC, "chunk table allocation failed");
    hipError_t e = hipMemcpy(cs.d_chunks, tab.data(), sizeof(Chunk) * tab.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(cs.d_chunks);
      return hip_fail(e, "chunk table upload");
    }
    if (dalloc(&cs.d_groups, groups.size()) != hipSuccess) {
      (void)hipFree(cs.d_chunks);
      return fail(GPE_ERR_ALLOC, "chunk group table allocation failed");
    }
    e = hipMemcpy(cs.d_groups, groups.data(), sizeof(GroupSegs) * groups.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(cs.d_chunks);
      (void)hipFree(cs.d_groups);
      return hip_fail(e, "chunk group table upload");
    }
    auto res = chunksets.emplace(key, std::move(cs));
    *out = &res.first->second;
    return GPE_OK;
  }

  // Order mode 4: workgroup b runs on XCD b % 8, so XCD x is given, plane
  // after plane, the x-th eighth of every x-plane's chunks.  The i-1 / i+1
  // neighbours of a site then lie in chunks the same XCD streamed just
  // before or will stream next (same L2), while all XCDs still work on the
  // same few planes at a time.  Which XCDs take the one-larger groups of a
  // plane rotates so the eight lists stay within one chunk of each other.
  gpe_status order_for(ChunkSet& cs, bool build = true) {
    if (cs.d_order) return GPE_OK;
    if (!build) return fail(GPE_ERR_STATE, "internal: the chunk order of the grid's launch variant is not built");
    std::vector<std::vector<int32_t>> lists(8);
    size_t c = 0;
    const size_t G = (size_t)cs.n_chunks;
    size_t pl = 0;
    while (c < G) {
      // chunks whose first site lies in the plane of chunk c
      while (pl + 1 < plane_begin.size() && plane_begin[pl + 1] <= cs.site_begin[c]) ++pl;
      const int64_t plane_end = (pl + 1 < plane_begin.size()) ? plane_begin[pl + 1] : INT64_MAX;
      size_t e = c;
      while (e < G && cs.site_begin[e] < plane_end) ++e;
      const size_t m = e - c, q = m / 8, r = m % 8;
      std::vector<int> by(8);
      for (int x = 0; x < 8; ++x) by[x] = x;
      std::stable_sort(by.begin(), by.end(), [&](int a, int b) { return lists[a].size() < lists[b].size(); });
      std::vector<char> big(8, 0);
      for (size_t k = 0; k < r; ++k) big[by[k]] = 1;
      for (int x = 0; x < 8; ++x) {
        const size_t take = q + (big[x] ? 1 : 0);
        for (size_t k = 0; k < take; ++k) lists[x].push_back((int32_t)(c++));
      }
      if (c != e) return fail(GPE_ERR_STATE, "internal: plane split of the chunk table");
    }
    // longer lists take the low XCD numbers so that b = 8 w + x < G covers them exactly
    std::stable_sort(lists.begin(), lists.end(),
                     [](const std::vector<int32_t>& a, const std::vector<int32_t>& b) { return a.size() > b.size(); });
    std::vector<int32_t> order(G);
    for (size_t b = 0; b < G; ++b) order[b] = lists[b % 8][b / 8];
    DeviceGuard g(device);
    if (dalloc(&cs.d_order, G) != hipSuccess) return fail(GPE_ERR_ALLOC, "chunk order allocation failed");
    hipError_t err = hipMemcpy(cs.d_order, order.data(), sizeof(int32_t) * G, hipMemcpyHostToDevice);
    if (err != hipSuccess) {
      (void)hipFree(cs.d_order);
      cs.d_order = nullptr;
      return hip_fail(err, "chunk order upload");
    }
    return GPE_OK;
  }

  Plan plan(const ChunkSet& cs, const LaunchConfig& cfg) const {
    Plan p;
    p.heads = stencil == 19 ? d_hoc_heads : (stencil == 27 ? d_c27_heads : d_heads);
    p.nbs = d_nbs;
    p.hoc = stencil == 7 ? 0 : stencil;
    p.hocnb = d_hoc_nbs;
    p.c27nb = d_c27_nbs;
    p.chunks = cs.d_chunks;
    p.groups = cs.d_groups;
    p.inst = d_inst;
    p.partials = d_partials;
    p.knot_acc = d_knot_acc;
    p.out = d_out;
    p.step = d_step;
    p.n_chunks = cs.n_chunks;
    p.n_inst = n_inst;
    p.xcd_map = cfg.xcd;
    p.order = cs.d_order;
    p.pstride = (int32_t)max_chunks;
    // complex128 is the widest per-site element (16 bytes)
    p.off32 = ((uint64_t)total * 16u < (uint64_t(1) << 32)) ? 1 : 0;
    p.max_seg = cs.max_seg;
    return p;
  }

  // Stream order across calls: work on stream s starts after the previous
  // call's work on this handle (whatever its stream) has ended.  Not applied
  // while s is being captured into a graph (the caller orders replays).
  gpe_status enter(hipStream_t s) {
    if (has_last && last_stream != s && !capturing(s))
      HIP_TRY(hipStreamWaitEvent(s, last_done, 0));
    return GPE_OK;
  }
  void leave(hipStream_t s) {
    if (capturing(s)) return;
    if (hipEventRecord(last_done, s) == hipSuccess) {
      last_stream = s;
      has_last = true;
    }
  }

  // Fill and upload the per-instance parameters.
  gpe_status upload(const ChunkSet& cs, const std::vector<InstParams>& ps, hipStream_t s) {
    return upload(cs, ps.data(), s);
  }
  gpe_status upload(const ChunkSet& cs, const InstParams* ps, hipStream_t s) {
    if (hipEventSynchronize(upload_done) != hipSuccess) return fail(GPE_ERR_DEVICE, "hipEventSynchronize failed");
    for (int i = 0; i < n_inst; ++i) {
      h_inst[i] = ps[i];
      h_inst[i].chunk_begin = cs.inst_begin[i];
      h_inst[i].chunk_count = cs.inst_count[i];
      h_inst[i].site_begin = inst_site[i];
      h_inst[i].n_sites = inst_site[i + 1] - inst_site[i];
      const double* h = &inst_h[3 * i];
      h_inst[i].cx = -0.5 / (h[0] * h[0]);
      h_inst[i].cy = -0.5 / (h[1] * h[1]);
      h_inst[i].cz = -0.5 / (h[2] * h[2]);
      h_inst[i].cd = 1.0 / (h[0] * h[0]) + 1.0 / (h[1] * h[1]) + 1.0 / (h[2] * h[2]);
      // eq. (B2): Lap_19 = Lap_7 + sum_{a<b} (h_a^2 + h_b^2)/12 delta_a^2 delta_b^2, as weights of -Lap/2
      const double h2[3] = {h[0] * h[0], h[1] * h[1], h[2] * h[2]};
      const double exy = (h2[0] + h2[1]) / (12.0 * h2[0] * h2[1]);
      const double exz = (h2[0] + h2[2]) / (12.0 * h2[0] * h2[2]);
      const double eyz = (h2[1] + h2[2]) / (12.0 * h2[1] * h2[2]);
      h_inst[i].qx = -0.5 * (1.0 / h2[0] - 2.0 * exy - 2.0 * exz);
      h_inst[i].qy = -0.5 * (1.0 / h2[1] - 2.0 * exy - 2.0 * eyz);
      h_inst[i].qz = -0.5 * (1.0 / h2[2] - 2.0 * exz - 2.0 * eyz);
      h_inst[i].qd = -0.5 * (-2.0 / h2[0] - 2.0 / h2[1] - 2.0 / h2[2] + 4.0 * (exy + exz + eyz));
      h_inst[i].qxy = -0.5 * exy;
      h_inst[i].qxz = -0.5 * exz;
      h_inst[i].qyz = -0.5 * eyz;
      h_inst[i].qc = 0.0;
      if (stencil == 27) {
        // cubic 27-point stencil for equal spacings: (1/(30 h^2)) [-128 centre,
        // 14 faces, 3 edges, 1 corners], as weights of -Lap/2
        const double u = -0.5 / (30.0 * h2[0]);
        h_inst[i].qd = -128.0 * u;
        h_inst[i].qx = h_inst[i].qy = h_inst[i].qz = 14.0 * u;
        h_inst[i].qxy = h_inst[i].qxz = h_inst[i].qyz = 3.0 * u;
        h_inst[i].qc = u;
      }
      h_inst[i].dV = h[0] * h[1] * h[2];
    }
    HIP_TRY(hipMemcpyAsync(d_inst, h_inst, sizeof(InstParams) * n_inst, hipMemcpyHostToDevice, s));
    HIP_TRY(hipEventRecord(upload_done, s));
    return GPE_OK;
  }
};

// Orders a call after the handle's previous call (Problem::enter) and marks
// its end on the call's stream when it goes out of scope (Problem::leave).
struct Ordered {
  Problem* P;
  hipStream_t s;
  gpe_status st;
  Ordered(Problem* p, hipStream_t st_) : P(p), s(st_) { st = P->enter(s); }
  ~Ordered() { P->leave(s); }
  Ordered(const Ordered&) = delete;
  Ordered& operator=(const Ordered&) = delete;
};

// work buffer carving (256-byte aligned sub-buffers)
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base((char*)b) {}
  void* take(size_t bytes) {
    void* p = base ? base + off : nullptr;
    off += (bytes + 255) & ~size_t(255);
    return p;
  }
};

// A host array that lives on the stack for up to 8 elements (a single grid's
// per-instance results), so the single-grid paths make no heap allocation.
template <typename T>
struct SmallBuf {
  T fixed[8];
  std::vector<T> big;
  T* p;
  explicit SmallBuf(size_t n) {
    if (n <= 8) {
      p = fixed;
    } else {
      big.resize(n);
      p = big.data();
    }
  }
  T& operator[](size_t i) { return p[i]; }
  T* data() { return p; }
};

size_t csize(int dtype) { return dtype == GPE_C128 ? 16 : 8; }
size_t rsize(int dtype) { return dtype == GPE_C128 ? 8 : 4; }

int64_t ckpt_interval(int64_t nsteps, int64_t ckpt_every) {
  if (ckpt_every > 0) return ckpt_every;
  int64_t k = (int64_t)std::ceil(std::sqrt((double)std::max<int64_t>(nsteps, 1)));
  while (k * k < nsteps) ++k;
  return std::max<int64_t>(k, 1);
}

// Memory-optimised tableaux of App. A (eqs. (A6)-(A7)): y^(i+1) = sum_j
// astar[i][j] y^(j) + dt asub[i] k_i and y_1 = sum_j bstar[j] y^(j) + dt bs k_s,
// k_i = f(t + c[i] dt, y^(i)); the coefficients are the ones printed there for
// Heun's third-order method and the fifth-order Cash-Karp weights.
struct MemOptTableau {
  int s;
  double c[6];
  double asub[6];
  double astar[6][6];
  double bstar[6];
  double bs;
};

const MemOptTableau kRKHE3 = {3,
                              {0.0, 1.0 / 3.0, 2.0 / 3.0},
                              {1.0 / 3.0, 2.0 / 3.0},
                              {{1.0}, {1.0, 0.0}},
                              {1.0 / 4.0, 3.0 / 4.0, 0.0},
                              3.0 / 4.0};

const MemOptTableau kRKCK = {6,
                             {0.0, 1.0 / 5.0, 3.0 / 10.0, 3.0 / 5.0, 1.0, 7.0 / 8.0},
                             {1.0 / 5.0, 9.0 / 40.0, 6.0 / 5.0, 35.0 / 27.0, 253.0 / 4096.0},
                             {{1.0},
                              {5.0 / 8.0, 3.0 / 8.0},
                              {2.0, 3.0, -4.0},
                              {-49.0 / 81.0, 35.0 / 27.0, 200.0 / 81.0, -175.0 / 81.0},
                              {253.0 / 12288.0, -3795.0 / 4096.0, 1375.0 / 1536.0, 2875.0 / 4096.0, 1265.0 / 4096.0}},
                             {-991.0 / 15939.0, -3865.0 / 5313.0, 5000.0 / 5313.0, 3125.0 / 4554.0, 25.0 / 154.0, 0.0},
                             512.0 / 1771.0};

const MemOptTableau* integrator_tableau(int integrator) {
  return integrator == GPE_RKHE3 ? &kRKHE3 : (integrator == GPE_RKCK ? &kRKCK : nullptr);
}

int rt_work_mode(int integrator) {
  return integrator == GPE_RKHE3 ? GPE_MODE_RT_RKHE3 : (integrator == GPE_RKCK ? GPE_MODE_RT_RKCK : GPE_MODE_RT);
}

int integrator_buffers(int integrator) {
  const MemOptTableau* t = integrator_tableau(integrator);
  return t ? t->s - 1 : 3;
}

size_t work_bytes_for(int64_t n, int dtype, int mode, int64_t nsteps, int64_t ckpt_every) {
  Carver c(nullptr);
  const size_t st = (size_t)n * csize(dtype);
  if (mode == GPE_MODE_ITP || mode == GPE_MODE_ITP_REAL) {
    // tmp, P and (19/27-point stencils) phi
    c.take(mode == GPE_MODE_ITP ? st : (size_t)n * rsize(dtype));
    c.take((size_t)n * rsize(dtype));
    c.take(mode == GPE_MODE_ITP ? st : (size_t)n * rsize(dtype));
  } else if (mode == GPE_MODE_RT || mode == GPE_MODE_RT_RKHE3 || mode == GPE_MODE_RT_RKCK) {
    const int integ = mode == GPE_MODE_RT ? GPE_RK4 : (mode == GPE_MODE_RT_RKHE3 ? GPE_RKHE3 : GPE_RKCK);
    for (int i = 0; i < integrator_buffers(integ); ++i) c.take(st);
  } else {
    // checkpoints + per segment step: state, Y2, Y3, Y4 + 8 vectors
    const int64_t K = ckpt_interval(nsteps, ckpt_every);
    const int64_t nck = (std::max<int64_t>(nsteps, 1) + K - 1) / K;
    for (int64_t i = 0; i < nck + 4 * K + 8; ++i) c.take(st);
  }
  return c.off;
}

}  // namespace

struct gpe_grid_s {
  Layout lay;
  int device = -1;
  int stencil = 7;          // selected stencil (also recorded for host-only grids)
  std::unique_ptr<Problem> prob;
  int64_t* d_run_base = nullptr;
  int32_t* d_run_start = nullptr;
  ~gpe_grid_s() {
    if (device >= 0) {
      DeviceGuard g(device);
      (void)hipFree(d_run_base);
      (void)hipFree(d_run_start);
    }
  }
};

struct gpe_batch_s {
  std::vector<gpe_grid> grids;
  int device = -1;
  std::unique_ptr<Problem> prob;
};

// ---------------------------------------------------------------------------
// validation helpers
// ---------------------------------------------------------------------------
namespace {

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

gpe_status check_dtype(int dtype) {
  if (dtype != GPE_C128 && dtype != GPE_C64) return fail(GPE_ERR_ARG, "dtype must be GPE_C128 or GPE_C64");
  return GPE_OK;
}

gpe_status check_ptr(const void* p, const char* name) {
  if (!p) return fail(GPE_ERR_ARG, "%s is NULL", name);
  if (!aligned16(p)) return fail(GPE_ERR_ARG, "%s is not 16-byte aligned", name);
  return GPE_OK;
}

gpe_status check_knots(int32_t n, const double* kt, const double* kv, const char* who) {
  if (n < 1 || n > GPE_MAX_KNOTS) return fail(GPE_ERR_ARG, "%s: n_knots must be in [1, %d]", who, GPE_MAX_KNOTS);
  if (!kt || !kv) return fail(GPE_ERR_ARG, "%s: knot arrays are NULL", who);
  for (int k = 0; k < n; ++k) {
    if (!std::isfinite(kt[k]) || !std::isfinite(kv[k])) return fail(GPE_ERR_ARG, "%s: non-finite knot", who);
    if (k > 0 && !(kt[k] > kt[k - 1])) return fail(GPE_ERR_ARG, "%s: knot_t must be strictly increasing", who);
  }
  return GPE_OK;
}

gpe_status check_pot(const gpe_potential* pot) {
  if (!pot) return fail(GPE_ERR_ARG, "potential is NULL");
  if (pot->kind != GPE_POT_STATIC && pot->kind != GPE_POT_RF_RAMP && pot->kind != GPE_POT_LERP &&
      pot->kind != GPE_POT_SHELL_RAMP)
    return fail(GPE_ERR_ARG, "unknown potential kind");
  gpe_status st = check_ptr(pot->field, "potential field");
  if (st != GPE_OK) return st;
  if (pot->kind == GPE_POT_LERP) {
    st = check_ptr(pot->field2, "potential field2");
    if (st != GPE_OK) return st;
    if (pot->n_knots != 2 || !pot->knot_t) return fail(GPE_ERR_ARG, "a LERP potential needs n_knots = 2 stage times");
    if (!std::isfinite(pot->knot_t[0]) || !std::isfinite(pot->knot_t[1]) || !(pot->knot_t[1] > pot->knot_t[0]))
      return fail(GPE_ERR_ARG, "LERP stage times must be finite and increasing");
    return GPE_OK;
  }
  if (pot->kind == GPE_POT_RF_RAMP || pot->kind == GPE_POT_SHELL_RAMP) {
    if (!std::isfinite(pot->omega)) return fail(GPE_ERR_ARG, "omega must be finite");
    return check_knots(pot->n_knots, pot->knot_t, pot->knot_delta, "potential");
  }
  return GPE_OK;
}

gpe_status check_params(const gpe_params* p) {
  if (!p) return fail(GPE_ERR_ARG, "params is NULL");
  if (!(p->dt > 0.0) || !std::isfinite(p->dt)) return fail(GPE_ERR_ARG, "dt must be finite and > 0");
  if (!std::isfinite(p->g)) return fail(GPE_ERR_ARG, "g must be finite");
  if (!std::isfinite(p->norm_target)) return fail(GPE_ERR_ARG, "norm_target must be finite");
  if (p->obs_every < 0) return fail(GPE_ERR_ARG, "obs_every must be >= 0");
  if (p->integrator != GPE_RK4 && p->integrator != GPE_RKHE3 && p->integrator != GPE_RKCK)
    return fail(GPE_ERR_ARG, "params.integrator must be GPE_RK4, GPE_RKHE3 or GPE_RKCK");
  return GPE_OK;
}

gpe_status check_grid(gpe_grid g) {
  if (!g) return fail(GPE_ERR_ARG, "grid is NULL");
  if (g->device < 0 || !g->prob) return fail(GPE_ERR_STATE, "grid is host-only (created with device -1)");
  return GPE_OK;
}

InstParams make_params(const gpe_potential* pot, const gpe_params* prm, double t0) {
  InstParams ip;
  std::memset(&ip, 0, sizeof ip);
  ip.g = prm ? prm->g : 0.0;
  ip.dt = prm ? prm->dt : 1.0;
  ip.t0 = t0;
  ip.norm_target = (prm && prm->norm_target > 0.0) ? prm->norm_target : 1.0;
  ip.pot_kind = pot ? pot->kind : GPE_POT_STATIC;
  const bool ramp = pot && (pot->kind == GPE_POT_RF_RAMP || pot->kind == GPE_POT_SHELL_RAMP);
  ip.omega = ramp ? pot->omega : 0.0;
  ip.n_knots = 1;
  ip.field2 = nullptr;
  if (pot && pot->kind == GPE_POT_LERP) {
    ip.n_knots = 2;
    ip.knot_t[0] = pot->knot_t[0];
    ip.knot_t[1] = pot->knot_t[1];
    ip.field2 = pot->field2;
  }
  if (ramp) {
    ip.n_knots = pot->n_knots;
    for (int k = 0; k < pot->n_knots; ++k) {
      ip.knot_t[k] = pot->knot_t[k];
      ip.knot_v[k] = pot->knot_delta[k];
    }
  }
  return ip;
}

// Gershgorin bound of the spectrum of T~: |centre| + sum |off-diagonal weights|
double kinetic_bound(const Problem& P) {
  double m = 0.0;
  for (int i = 0; i < P.n_inst; ++i) {
    const double* h = &P.inst_h[3 * i];
    const double h2[3] = {h[0] * h[0], h[1] * h[1], h[2] * h[2]};
    if (P.stencil == 27) {
      m = std::max(m, 128.0 / (30.0 * h2[0]));
    } else if (P.stencil == 19) {
      const double exy = (h2[0] + h2[1]) / (12.0 * h2[0] * h2[1]);
      const double exz = (h2[0] + h2[2]) / (12.0 * h2[0] * h2[2]);
      const double eyz = (h2[1] + h2[2]) / (12.0 * h2[1] * h2[2]);
      const double fx = std::fabs(1.0 / h2[0] - 2.0 * exy - 2.0 * exz);
      const double fy = std::fabs(1.0 / h2[1] - 2.0 * exy - 2.0 * eyz);
      const double fz = std::fabs(1.0 / h2[2] - 2.0 * exz - 2.0 * eyz);
      const double c = std::fabs(-2.0 / h2[0] - 2.0 / h2[1] - 2.0 / h2[2] + 4.0 * (exy + exz + eyz));
      m = std::max(m, 0.5 * (c + 2.0 * (fx + fy + fz) + 4.0 * (exy + exz + eyz)));
    } else {
      m = std::max(m, 2.0 * (1.0 / h2[0] + 1.0 / h2[1] + 1.0 / h2[2]));
    }
  }
  return m;
}

// ---------------------------------------------------------------------------
// drivers
// ---------------------------------------------------------------------------
struct Ctx {
  Problem* P;
  ChunkSet* cs;
  LaunchConfig cfg;
  Plan pl;
  hipStream_t s;
};

gpe_status make_ctx(Problem* P, int config, hipStream_t s, Ctx& c, bool build = true) {
  c.P = P;
  c.cfg = config_get(config);
  const bool hoc = P->stencil != 7;
  if ((uint64_t)P->total * 16u >= (uint64_t(1) << 32)) {
    if (hoc) return fail(GPE_ERR_ARG, "the 19- and 27-point stencils need arrays below 4 GiB");
    // 64-bit addressing is compiled for one shape only
    c.cfg.block = 256;
    c.cfg.spt = 2;
    c.cfg.nt = 0;
    c.cfg.stage = 1;
  }
  if (hoc) {
    // the 19-point kernels are compiled for 256 lanes x 1 site
    c.cfg.block = 256;
    c.cfg.spt = 1;
    c.cfg.stage = 1;
  }
  gpe_status st = P->chunks_for(chunk_capacity(c.cfg), &c.cs, P->stencil, build);
  if (st != GPE_OK) return st;
  if (c.cfg.xcd == 4) {
    st = P->order_for(*c.cs, build);
    if (st != GPE_OK) return st;
  }
  c.pl = P->plan(*c.cs, c.cfg);
  c.s = s;
  return GPE_OK;
}

// Build the chunk table (and chunk order) of the problem's current launch
// variant and stencil now, so that calls on it allocate no device memory
// (grid creation and every change of variant or stencil do this).
gpe_status prepare_tables(Problem* P) {
  Ctx c;
  return make_ctx(P, P->config, nullptr, c, true);
}

#define LTRY(expr)                                          \
  do {                                                      \
    hipError_t _e = (expr);                                 \
    if (_e != hipSuccess) return hip_fail(_e, #expr);       \
  } while (0)

// One RK4 step n (step < 0: the step index is read from the device counter,
// which is then advanced; used for captured graphs).
// Scratch buffers b1, b2, b3 (each one state vector).  Scheme 0 keeps y2, y3,
// y4 in b1, b2, b3; scheme 1 keeps y2 in b1, y3 in b2, A in b3 and writes y4
// over y2 (b1) once stage 2 has folded y2 into A.
template <typename R>
gpe_status rk_step(const Ctx& c, const void* y0, const void* field, void* b1, void* b2, void* b3, void* out,
                   bool obs, gpe_obs* obs_dev, int64_t step) {
  LTRY(run_rk_stage<R>(c.pl, c.cfg, 1, obs, y0, y0, nullptr, nullptr, field, b1, step, c.s));
  if (obs) LTRY(run_finalize(c.pl, FIN_OBS, obs_dev, c.s));
  if (c.cfg.scheme == 1) {
    LTRY(run_rk_stage2_fold<R>(c.pl, c.cfg, b1, y0, field, b2, b3, step, c.s));
    LTRY(run_rk_stage<R>(c.pl, c.cfg, 3, false, b2, y0, nullptr, nullptr, field, b1, step, c.s));
    LTRY(run_rk_stage4_fold<R>(c.pl, c.cfg, b1, b3, field, out, step, c.s));
  } else {
    LTRY(run_rk_stage<R>(c.pl, c.cfg, 2, false, b1, y0, nullptr, nullptr, field, b2, step, c.s));
    LTRY(run_rk_stage<R>(c.pl, c.cfg, 3, false, b2, y0, nullptr, nullptr, field, b3, step, c.s));
    LTRY(run_rk_stage<R>(c.pl, c.cfg, 4, false, b3, y0, b1, b2, field, out, step, c.s));
  }
  if (step < 0) LTRY(run_tick(c.pl.step, 1, c.s));
  return GPE_OK;
}

// One step of a memory-optimised method: Y[0] = y0 (in/out), Y[1..s-1] scratch.
template <typename R>
gpe_status rk_generic_step(const Ctx& c, const MemOptTableau& tb, void* y0, const void* field, void* const* buf,
                           int64_t step) {
  void* Y[6];
  Y[0] = y0;
  for (int i = 1; i < tb.s; ++i) Y[i] = buf[i - 1];
  for (int i = 0; i < tb.s; ++i) {
    const bool final_stage = (i == tb.s - 1);
    const double* row = final_stage ? tb.bstar : tb.astar[i];
    // coefficient of the stencil input y^(i) itself, then the earlier states
    const double ccur = row[i];
    const void* hist[6];
    double hc[6];
    int nh = 0;
    for (int j = 0; j < i; ++j)
      if (row[j] != 0.0) {
        hist[nh] = Y[j];
        hc[nh] = row[j];
        ++nh;
      }
    const double cdt = final_stage ? tb.bs : tb.asub[i];
    void* out = final_stage ? y0 : Y[i + 1];
    LTRY(run_rk_generic<R>(c.pl, c.cfg, Y[i], ccur, nh, hist, hc, cdt, tb.c[i], field, out, step, c.s));
  }
  if (step < 0) LTRY(run_tick(c.pl.step, 1, c.s));
  return GPE_OK;
}

// instances of at most this many chunks form the imaginary-time scale inside
// the next pass instead of a finalize launch
constexpr int kFuseScaleChunks = 1024;

template <typename R>
gpe_status drive_itp(const Ctx& c, void* psi, const void* field, int64_t nsteps, void* work, int64_t obs_every,
                     gpe_obs* hist, bool real = false) {
  Carver cv(work);
  void* tmp = cv.take((size_t)c.P->total * (real ? 1 : 2) * sizeof(R));
  void* prop = cv.take((size_t)c.P->total * sizeof(R));
  // With the 19/27-point stencils the first pass would apply the diagonal
  // half-step at every one of 16/24 lateral taps (two gathers each); a
  // separate site-by-site pass forms phi once instead.
  const bool split_diag = c.P->stencil != 7;
  void* phi = split_diag ? cv.take((size_t)c.P->total * (real ? 1 : 2) * sizeof(R)) : nullptr;
  LTRY(run_set_step(c.pl.step, 0, c.s));
  LTRY(run_make_prop<R>(c.pl, c.cfg, field, prop, c.s));
  LTRY(run_set_scale_one(c.pl, c.s));
  // On small grids, where launches rather than bytes set the pace, pass 1
  // forms the scale from pass 2's norm partials itself and the finalize runs
  // after the last step only (the observations read the stored scale, so a
  // run with a history keeps the finalize).
  int max_chunks = 0;
  for (int q : c.cs->inst_count) max_chunks = std::max(max_chunks, q);
  const bool fuse = !split_diag && !(hist && obs_every > 0) && max_chunks <= kFuseScaleChunks;
  int64_t k = 0;
  for (int64_t n = 0; n < nsteps; ++n) {
    if (hist && obs_every > 0 && n % obs_every == 0) {
      LTRY(run_observe<R>(c.pl, c.cfg, psi, field, 0.0, true, 0, c.s, real));
      LTRY(run_finalize(c.pl, FIN_OBS, hist + k * c.P->n_inst, c.s));
      ++k;
    }
    if (split_diag) {
      LTRY(run_itp_phi<R>(c.pl, c.cfg, psi, prop, phi, real, c.s));
      LTRY(run_itp_pass1<R>(c.pl, c.cfg, phi, prop, tmp, real, c.s, true));
    } else {
      LTRY(run_itp_pass1<R>(c.pl, c.cfg, psi, prop, tmp, real, c.s, false, fuse && n > 0));
    }
    LTRY(run_itp_pass2<R>(c.pl, c.cfg, tmp, prop, psi, real, c.s));
    if (!fuse || n == nsteps - 1) LTRY(run_finalize(c.pl, FIN_NORM_SCALE, nullptr, c.s));
  }
  if (nsteps > 0) LTRY(run_apply_scale<R>(c.pl, c.cfg, psi, real, c.s));
  return GPE_OK;
}

template <typename R>
gpe_status drive_rt(const Ctx& c, void* psi, const void* field, int64_t nsteps, void* work, int64_t obs_every,
                    gpe_obs* hist, int integrator = GPE_RK4) {
  Carver cv(work);
  const size_t st = (size_t)c.P->total * 2 * sizeof(R);
  const MemOptTableau* tb = integrator_tableau(integrator);
  if (tb) {
    void* buf[5];
    for (int i = 0; i < tb->s - 1; ++i) buf[i] = cv.take(st);
    int64_t k = 0;
    for (int64_t n = 0; n < nsteps; ++n) {
      if (hist && obs_every > 0 && n % obs_every == 0) {
        LTRY(run_observe<R>(c.pl, c.cfg, psi, field, 0.0, false, n, c.s));
        LTRY(run_finalize(c.pl, FIN_OBS, hist + k * c.P->n_inst, c.s));
        ++k;
      }
      gpe_status r = rk_generic_step<R>(c, *tb, psi, field, buf, n);
      if (r != GPE_OK) return r;
    }
    return GPE_OK;
  }
  void* y2 = cv.take(st);
  void* y3 = cv.take(st);
  void* y4 = cv.take(st);
  int64_t k = 0;
  for (int64_t n = 0; n < nsteps; ++n) {
    const bool obs = hist && obs_every > 0 && n % obs_every == 0;
    gpe_status r = rk_step<R>(c, psi, field, y2, y3, y4, psi, obs, obs ? hist + k * c.P->n_inst : nullptr, n);
    if (r != GPE_OK) return r;
    if (obs) ++k;
  }
  return GPE_OK;
}

template <typename R>
gpe_status drive_observe(const Ctx& c, const void* psi, const void* field, bool use_scale, int64_t step,
                         bool real = false) {
  LTRY(run_observe<R>(c.pl, c.cfg, psi, field, 0.0, use_scale, step, c.s, real));
  LTRY(run_finalize(c.pl, FIN_OBS, nullptr, c.s));
  return GPE_OK;
}

gpe_status read_obs(Problem& P, gpe_obs* out_host, hipStream_t s) {
  SmallBuf<InstOut> o(P.n_inst);
  HIP_TRY(hipMemcpyAsync(o.data(), P.d_out, sizeof(InstOut) * P.n_inst, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  bool finite = true;
  for (int i = 0; i < P.n_inst; ++i) {
    out_host[i].norm = o[i].norm;
    out_host[i].energy = o[i].energy;
    out_host[i].mu = o[i].mu;
    finite = finite && std::isfinite(o[i].norm) && std::isfinite(o[i].energy);
  }
  if (!finite) return fail(GPE_ERR_NONFINITE, "observed norm/energy is not finite");
  return GPE_OK;
}

// adjoint: loss and knot gradients, fully on the device
constexpr size_t kMaxGraphs = 16;

// Captured graph of one in-place RK4 step of psi (scratch y2, y3, y4); the
// step index comes from the device counter, so one graph serves every step.
template <typename R>
static gpe_status step_graph(const Ctx& c, int dtype, void* psi, const void* field, int integrator,
                             void* const* bufs, hipGraphExec_t* out) {
  Problem& P = *c.P;
  Problem::GraphKey key{psi, field, bufs[0], dtype, P.config, c.cfg.scheme, integrator, P.stencil};
  auto it = P.graphs.find(key);
  if (it != P.graphs.end()) {
    *out = it->second;
    return GPE_OK;
  }
  hipGraphExec_t exec = nullptr;
  hipStream_t cap = nullptr;
  HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  gpe_status r = GPE_OK;
  if (e == hipSuccess) {
    Ctx cc = c;
    cc.s = cap;
    const MemOptTableau* tb = integrator_tableau(integrator);
    r = tb ? rk_generic_step<R>(cc, *tb, psi, field, bufs, -1)
           : rk_step<R>(cc, psi, field, bufs[0], bufs[1], bufs[2], psi, false, nullptr, -1);
    hipError_t e2 = hipStreamEndCapture(cap, &graph);
    if (r == GPE_OK && e2 != hipSuccess) r = hip_fail(e2, "hipStreamEndCapture");
  } else {
    r = hip_fail(e, "hipStreamBeginCapture");
  }
  if (r == GPE_OK) {
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) r = hip_fail(e, "hipGraphInstantiate");
  }
  if (graph) (void)hipGraphDestroy(graph);
  (void)hipStreamDestroy(cap);
  if (r != GPE_OK) return r;
  // a caller that cycles through many buffers would otherwise keep one
  // instantiated graph per buffer set for the life of the grid
  if (P.graphs.size() >= kMaxGraphs) {
    HIP_TRY(hipDeviceSynchronize());     // none of them may still be running
    for (auto& kv : P.graphs) (void)hipGraphExecDestroy(kv.second);
    P.graphs.clear();
  }
  P.graphs[key] = exec;
  *out = exec;
  return GPE_OK;
}

// Discrete adjoint of the RK4 map with checkpointing: the forward sweep keeps
// every K-th state (K = ceil(sqrt(nsteps)) by default); the reverse sweep
// recomputes each segment of K steps from its checkpoint, keeping the stage
// states Y2, Y3, Y4 of every step of the segment, then runs the four adjoint
// stages of each step in reverse.  The whole driver uses the App. A storage
// scheme (distinct y2, y3, y4), so recomputed states equal the forward
// sweep's bit for bit.  use_graph: the forward sweep replays a captured step
// graph (the checkpoint copies run eagerly between replays).
template <typename R>
gpe_status drive_adjoint(const Ctx& c_in, const void* psi0, const void* target, const void* field, int64_t nsteps,
                         int64_t ckpt_every, void* work, void* psi_final, bool use_graph = false) {
  Ctx c = c_in;
  c.cfg.scheme = 0;
  const int64_t K = ckpt_interval(nsteps, ckpt_every);
  const int64_t nck = (std::max<int64_t>(nsteps, 1) + K - 1) / K;
  const size_t st = (size_t)c.P->total * 2 * sizeof(R);
  Carver cv(work);
  std::vector<void*> ck(nck), seg(K), s2(K), s3(K), s4(K);
  for (auto& p : ck) p = cv.take(st);
  for (int64_t r = 0; r < K; ++r) {
    seg[r] = cv.take(st);
    s2[r] = cv.take(st);
    s3[r] = cv.take(st);
    s4[r] = cv.take(st);
  }
  void* y2 = cv.take(st);
  void* y3 = cv.take(st);
  void* y4 = cv.take(st);
  void* lam = cv.take(st);
  void* lacc = cv.take(st);
  void* uA = cv.take(st);
  void* uB = cv.take(st);
  void* cur = cv.take(st);

  LTRY(hipMemcpyAsync(cur, psi0, st, hipMemcpyDeviceToDevice, c.s));
  hipGraphExec_t fwd = nullptr;
  if (use_graph) {
    void* bufs[3] = {y2, y3, y4};
    gpe_status r = step_graph<R>(c, sizeof(R) == 8 ? GPE_C128 : GPE_C64, cur, field, GPE_RK4, bufs, &fwd);
    if (r != GPE_OK) return r;
    LTRY(run_set_step(c.pl.step, 0, c.s));
  }
  for (int64_t n = 0; n < nsteps; ++n) {
    if (n % K == 0) LTRY(hipMemcpyAsync(ck[n / K], cur, st, hipMemcpyDeviceToDevice, c.s));
    if (fwd) {
      LTRY(hipGraphLaunch(fwd, c.s));
    } else {
      gpe_status r = rk_step<R>(c, cur, field, y2, y3, y4, cur, false, nullptr, n);
      if (r != GPE_OK) return r;
    }
  }
  if (psi_final) LTRY(hipMemcpyAsync(psi_final, cur, st, hipMemcpyDeviceToDevice, c.s));
  LTRY(run_overlap<R>(c.pl, c.cfg, target, cur, c.s));
  LTRY(run_finalize(c.pl, FIN_OVERLAP, nullptr, c.s));
  LTRY(run_finalize(c.pl, FIN_LOSS, nullptr, c.s));
  LTRY(run_seed_lambda<R>(c.pl, c.cfg, target, lam, c.s));
  LTRY(run_zero_doubles(c.pl.knot_acc, (int64_t)c.cs->n_chunks * GPE_MAX_KNOTS, c.s));
  for (int64_t m = nck - 1; m >= 0; --m) {
    const int64_t n0 = m * K, L = std::min(K, nsteps - n0);
    void* Y1 = ck[m];
    for (int64_t r = 0; r < L; ++r) {
      const int64_t n = n0 + r;
      LTRY(run_rk_stage<R>(c.pl, c.cfg, 1, false, Y1, Y1, nullptr, nullptr, field, s2[r], n, c.s));
      LTRY(run_rk_stage<R>(c.pl, c.cfg, 2, false, s2[r], Y1, nullptr, nullptr, field, s3[r], n, c.s));
      LTRY(run_rk_stage<R>(c.pl, c.cfg, 3, false, s3[r], Y1, nullptr, nullptr, field, s4[r], n, c.s));
      if (r + 1 < L) {
        LTRY(run_rk_stage<R>(c.pl, c.cfg, 4, false, s4[r], Y1, s2[r], s3[r], field, seg[r + 1], n, c.s));
        Y1 = seg[r + 1];
      }
    }
    for (int64_t r = L - 1; r >= 0; --r) {
      const int64_t n = n0 + r;
      void* Yr = r == 0 ? ck[m] : seg[r];
      LTRY(run_adj_stage<R>(c.pl, c.cfg, 4, lam, s4[r], field, nullptr, lacc, uA, n, c.s));
      LTRY(run_adj_stage<R>(c.pl, c.cfg, 3, uA, s3[r], field, lam, lacc, uB, n, c.s));
      LTRY(run_adj_stage<R>(c.pl, c.cfg, 2, uB, s2[r], field, lam, lacc, uA, n, c.s));
      LTRY(run_adj_stage<R>(c.pl, c.cfg, 1, uA, Yr, field, nullptr, lacc, lam, n, c.s));
    }
  }
  LTRY(run_knot_finalize(c.pl, c.P->d_grads, c.s));
  return GPE_OK;
}

gpe_status read_loss_grad(Problem& P, double* loss_host, double* grad_host, int n_knots_single) {
  std::vector<InstOut> o(P.n_inst);
  std::vector<double> gr((size_t)P.n_inst * GPE_MAX_KNOTS);
  HIP_TRY(hipMemcpy(o.data(), P.d_out, sizeof(InstOut) * P.n_inst, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(gr.data(), P.d_grads, sizeof(double) * gr.size(), hipMemcpyDeviceToHost));
  bool finite = true;
  for (int i = 0; i < P.n_inst; ++i) {
    if (loss_host) loss_host[i] = o[i].loss;
    finite = finite && std::isfinite(o[i].loss);
  }
  if (grad_host) {
    if (n_knots_single > 0) {
      for (int k = 0; k < n_knots_single; ++k) grad_host[k] = gr[k];
    } else {
      std::memcpy(grad_host, gr.data(), sizeof(double) * gr.size());
    }
  }
  if (!finite) return fail(GPE_ERR_NONFINITE, "loss is not finite");
  return GPE_OK;
}

// Per-instance bounds for the stability checks, from one device pass over the
// potential field and the state: vmax[i] bounds |V| over the call's time span
// (for an RF ramp |V| <= sqrt(max_k |U - Delta_k|^2 + omega^2) over the knots
// Delta_k, since Delta(t) stays between knot values; for a stage
// interpolation the larger of the two arrays' bounds), dmax[i] is the largest
// |psi|^2 of the start state.
template <typename R>
gpe_status field_bounds(const Ctx& c, const void* field, const void* psi, bool real_psi, const InstParams* ps,
                        double* vmax, double* dmax) {
  const int n = c.P->n_inst;
  LTRY(run_field_range<R>(c.pl, c.cfg, field, psi, c.s, real_psi));
  LTRY(run_finalize(c.pl, FIN_RANGE, nullptr, c.s));
  SmallBuf<InstOut> o(n);
  HIP_TRY(hipMemcpyAsync(o.data(), c.P->d_out, sizeof(InstOut) * n, hipMemcpyDeviceToHost, c.s));
  HIP_TRY(hipStreamSynchronize(c.s));
  for (int i = 0; i < n; ++i) {
    vmax[i] = 0.0;
    dmax[i] = 0.0;
  }
  for (int i = 0; i < n; ++i) {
    const InstParams& ip = ps[i];
    dmax[i] = o[i].dmax;
    if (ip.pot_kind == GPE_POT_RF_RAMP || ip.pot_kind == GPE_POT_SHELL_RAMP) {
      // the ramp parameter stays between knot values, where |field - it| is
      // largest at an end of the field's range
      for (int k = 0; k < ip.n_knots; ++k) {
        const double d = std::max(std::fabs(o[i].fmax - ip.knot_v[k]), std::fabs(o[i].fmin - ip.knot_v[k]));
        const double v = ip.pot_kind == GPE_POT_SHELL_RAMP ? 0.5 * std::fabs(ip.omega) * d * d
                                                           : std::sqrt(d * d + ip.omega * ip.omega);
        vmax[i] = std::max(vmax[i], v);
      }
    } else {
      vmax[i] = std::max(std::fabs(o[i].fmin), std::fabs(o[i].fmax));
    }
  }
  if (n == 1 && ps[0].pot_kind == GPE_POT_LERP) {
    // V is a convex combination of the two stage arrays
    LTRY(run_field_range<R>(c.pl, c.cfg, ps[0].field2, nullptr, c.s));
    LTRY(run_finalize(c.pl, FIN_RANGE, nullptr, c.s));
    HIP_TRY(hipMemcpyAsync(o.data(), c.P->d_out, sizeof(InstOut), hipMemcpyDeviceToHost, c.s));
    HIP_TRY(hipStreamSynchronize(c.s));
    vmax[0] = std::max(vmax[0], std::max(std::fabs(o[0].fmin), std::fabs(o[0].fmax)));
  }
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(vmax[i]) || !std::isfinite(dmax[i]))
      return fail(GPE_ERR_NONFINITE, "instance %d: the potential or the start state is not finite", i);
  return GPE_OK;
}

}  // namespace

// Stability of an explicit real-time step (default on; params.skip_stability_check
// opts out).  For every instance the spectrum of the frozen-coefficient
// operator T~ + V + g|psi|^2 of eq. (8) is bounded by Gershgorin:
// lambda = lambda(T~) + max|V| + gfac |g| max|psi|^2 (gfac = 1; the fidelity
// gradient's linearised operator (T~ + V + 2g|Y|^2) u + g Y^2 conj(u) takes
// gfac = 3), and dt lambda must stay inside the method's stability interval
// on the imaginary axis: 2 sqrt 2 for RK4, sqrt 3 for any three-stage
// third-order method.  The Cash-Karp fifth-order weights have |R(iy)| = 1 +
// y^6/7200 + O(y^8) > 1 for every y, so no step is strictly stable; the check
// then caps dt lambda at 1, where the spurious growth per step stays below
// 2.3e-4.  max|psi|^2 is that of the start state.
template <typename R>
static gpe_status rt_stability(const Ctx& c, const InstParams* ps, const void* field, const void* psi,
                               int integrator = GPE_RK4, double gfac = 1.0) {
  SmallBuf<double> vmax(c.P->n_inst), dmax(c.P->n_inst);
  gpe_status st = field_bounds<R>(c, field, psi, false, ps, vmax.data(), dmax.data());
  if (st != GPE_OK) return st;
  const double kin = kinetic_bound(*c.P);
  const double bound = integrator == GPE_RKHE3 ? std::sqrt(3.0) : (integrator == GPE_RKCK ? 1.0 : 2.0 * std::sqrt(2.0));
  for (int i = 0; i < c.P->n_inst; ++i) {
    const double lam = kin + vmax[i] + gfac * std::fabs(ps[i].g) * dmax[i];
    if (ps[i].dt * lam > bound)
      return fail(GPE_ERR_UNSTABLE,
                  "instance %d: dt = %g exceeds the stability bound %g/lambda = %g (lambda = %g: kinetic %g, max V %g, "
                  "%g g max|psi|^2 %g)",
                  i, ps[i].dt, bound, bound / lam, lam, kin, vmax[i], gfac, std::fabs(ps[i].g) * dmax[i]);
  }
  return GPE_OK;
}

// Stability of the imaginary-time step: each forward-Euler kinetic substep of
// dt/2 needs (dt/2) lambda(T~) <= 2, and the linearised interaction factor
// 1 - g|psi|^2 dt/2 of the diagonal half-step must stay positive at the start
// state.
template <typename R>
static gpe_status itp_stability(const Ctx& c, const InstParams* ps, const void* field, const void* psi,
                                bool real) {
  const double lt = kinetic_bound(*c.P);
  for (int i = 0; i < c.P->n_inst; ++i)
    if (ps[i].dt * lt > 4.0)
      return fail(GPE_ERR_UNSTABLE, "dt = %g exceeds the Euler-substep bound 4/lambda_T = %g", ps[i].dt, 4.0 / lt);
  SmallBuf<double> vmax(c.P->n_inst), dmax(c.P->n_inst);
  gpe_status st = field_bounds<R>(c, field, psi, real, ps, vmax.data(), dmax.data());
  if (st != GPE_OK) return st;
  for (int i = 0; i < c.P->n_inst; ++i)
    if (ps[i].g * dmax[i] * ps[i].dt * 0.5 >= 1.0)
      return fail(GPE_ERR_UNSTABLE,
                  "dt = %g makes the interaction factor 1 - g|psi|^2 dt/2 non-positive (g max|psi|^2 = %g)", ps[i].dt,
                  ps[i].g * dmax[i]);
  return GPE_OK;
}

template <typename R>
static gpe_status batch_rt_graph(const Ctx& c, int dtype, void* psi, const void* field, int64_t nsteps, void* work,
                                 int integrator) {
  Carver cv(work);
  const size_t st = (size_t)c.P->total * 2 * sizeof(R);
  void* bufs[5];
  for (int i = 0; i < integrator_buffers(integrator); ++i) bufs[i] = cv.take(st);
  hipGraphExec_t exec = nullptr;
  gpe_status r = step_graph<R>(c, dtype, psi, field, integrator, bufs, &exec);
  if (r != GPE_OK) return r;
  HIP_TRY(run_set_step(c.pl.step, 0, c.s));
  for (int64_t n = 0; n < nsteps; ++n) HIP_TRY(hipGraphLaunch(exec, c.s));
  return GPE_OK;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* gpe_last_error(void) { return t_err.c_str(); }
int gpe_abi_version(void) { return GPE_ABI_VERSION; }

static gpe_status finish_grid(const gpe_geometry* geom, Layout&& lay, int device, gpe_grid* out) {
  for (int d = 0; d < 3; ++d) {
    lay.h[d] = geom->h[d];
    lay.x0[d] = geom->x0[d];
  }
  gpe_grid g = new (std::nothrow) gpe_grid_s();
  if (!g) return fail(GPE_ERR_ALLOC, "out of host memory");
  g->lay = std::move(lay);
  g->device = device;
  if (device >= 0) {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device >= ndev) {
      delete g;
      return fail(GPE_ERR_DEVICE, "device %d not available", device);
    }
    g->prob.reset(new (std::nothrow) Problem());
    if (!g->prob) {
      delete g;
      return fail(GPE_ERR_ALLOC, "out of host memory");
    }
    std::vector<const Layout*> lays{&g->lay};
    gpe_status st = g->prob->build(device, lays);
    if (st == GPE_OK) {
      DeviceGuard dg(device);
      st = prepare_tables(g->prob.get());
    }
    if (st != GPE_OK) {
      g->device = -1;
      delete g;
      return st;
    }
    DeviceGuard dg(device);
    const Layout& L = g->lay;
    const int64_t nr = L.n_runs();
    std::vector<int64_t> base(nr);
    std::vector<int32_t> start(nr);
    for (int64_t r = 0; r < nr; ++r) {
      base[r] = (L.run_i[r] * L.n[1] + L.run_j[r]) * L.n[2] + L.run_k0[r];
      start[r] = (int32_t)L.run_start[r];
    }
    if (dalloc(&g->d_run_base, nr) != hipSuccess || dalloc(&g->d_run_start, nr) != hipSuccess ||
        hipMemcpy(g->d_run_base, base.data(), sizeof(int64_t) * nr, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(g->d_run_start, start.data(), sizeof(int32_t) * nr, hipMemcpyHostToDevice) != hipSuccess) {
      delete g;
      return fail(GPE_ERR_ALLOC, "run table allocation/upload failed");
    }
  }
  *out = g;
  return GPE_OK;
}

static gpe_status check_geom(const gpe_geometry* geom) {
  if (!geom) return fail(GPE_ERR_ARG, "geometry is NULL");
  for (int d = 0; d < 3; ++d) {
    if (geom->n[d] < 1) return fail(GPE_ERR_ARG, "geometry: n[%d] must be >= 1", d);
    if (!(geom->h[d] > 0.0) || !std::isfinite(geom->h[d])) return fail(GPE_ERR_ARG, "geometry: h[%d] must be > 0", d);
    if (!std::isfinite(geom->x0[d])) return fail(GPE_ERR_ARG, "geometry: x0[%d] must be finite", d);
  }
  return GPE_OK;
}

gpe_status gpe_grid_create(const gpe_geometry* geom, const uint8_t* mask_host, int device, gpe_grid* out) {
  if (!out) return fail(GPE_ERR_ARG, "out is NULL");
  *out = nullptr;
  gpe_status st = check_geom(geom);
  if (st != GPE_OK) return st;
  if (!mask_host) return fail(GPE_ERR_ARG, "mask is NULL");
  if (device < -1) return fail(GPE_ERR_ARG, "device must be >= -1");
  Layout lay;
  std::string err = layout_from_mask(geom->n, mask_host, lay);
  if (!err.empty()) return fail(GPE_ERR_ARG, "%s", err.c_str());
  return finish_grid(geom, std::move(lay), device, out);
}

gpe_status gpe_grid_create_runs(const gpe_geometry* geom, int64_t nruns, const int64_t* runs_host, int device,
                                gpe_grid* out) {
  if (!out) return fail(GPE_ERR_ARG, "out is NULL");
  *out = nullptr;
  gpe_status st = check_geom(geom);
  if (st != GPE_OK) return st;
  if (!runs_host || nruns < 1) return fail(GPE_ERR_ARG, "runs must be non-empty");
  if (device < -1) return fail(GPE_ERR_ARG, "device must be >= -1");
  Layout lay;
  std::string err = layout_from_runs(geom->n, nruns, runs_host, lay);
  if (!err.empty()) return fail(GPE_ERR_ARG, "%s", err.c_str());
  return finish_grid(geom, std::move(lay), device, out);
}

gpe_status gpe_grid_create_threshold(const gpe_geometry* geom, gpe_dtype dtype, const void* va_box,
                                     const void* vb_box, double cutoff, int device, gpe_grid* out) {
  if (!out) return fail(GPE_ERR_ARG, "out is NULL");
  *out = nullptr;
  gpe_status st = check_geom(geom);
  if (st == GPE_OK) st = check_dtype(dtype);
  if (st == GPE_OK) st = check_ptr(va_box, "va_box");
  if (st != GPE_OK) return st;
  if (vb_box) {
    st = check_ptr(vb_box, "vb_box");
    if (st != GPE_OK) return st;
  }
  if (std::isnan(cutoff)) return fail(GPE_ERR_ARG, "cutoff is NaN");
  if (device < 0) return fail(GPE_ERR_ARG, "the potentials live on a device: device must be >= 0");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device >= ndev) return fail(GPE_ERR_DEVICE, "device %d not available", device);
  // the z-runs of the selection are found on the device (a count pass, the
  // column offsets, an emit pass); only the run table comes to the host
  const int64_t n0 = geom->n[0], n1 = geom->n[1], n2 = geom->n[2], n01 = n0 * n1;
  std::vector<int64_t> runs;
  {
    DeviceGuard dg(device);
    if (!dg.ok) return fail(GPE_ERR_DEVICE, "hipSetDevice(%d) failed", device);
    auto column_runs = [&](int32_t* cnt, const int64_t* off, int64_t* rr) {
      return dtype == GPE_C128 ? run_column_runs<double>(va_box, vb_box, n0, n1, n2, cutoff, cnt, off, rr, nullptr)
                               : run_column_runs<float>(va_box, vb_box, n0, n1, n2, cutoff, cnt, off, rr, nullptr);
    };
    int32_t* d_cnt = nullptr;
    int64_t* d_off = nullptr;
    int64_t* d_runs = nullptr;
    std::vector<int32_t> cnt((size_t)n01);
    std::vector<int64_t> off((size_t)n01);
    hipError_t e = hipMalloc((void**)&d_cnt, sizeof(int32_t) * (size_t)n01);
    if (e == hipSuccess) e = column_runs(d_cnt, nullptr, nullptr);
    if (e == hipSuccess) e = hipMemcpy(cnt.data(), d_cnt, sizeof(int32_t) * (size_t)n01, hipMemcpyDeviceToHost);
    int64_t total = 0;
    if (e == hipSuccess) {
      for (int64_t c = 0; c < n01; ++c) {
        off[(size_t)c] = total;
        total += cnt[(size_t)c];
      }
    }
    if (e == hipSuccess && total > 0) {
      e = hipMalloc((void**)&d_off, sizeof(int64_t) * (size_t)n01);
      if (e == hipSuccess) e = hipMalloc((void**)&d_runs, sizeof(int64_t) * 4 * (size_t)total);
      if (e == hipSuccess) e = hipMemcpy(d_off, off.data(), sizeof(int64_t) * (size_t)n01, hipMemcpyHostToDevice);
      if (e == hipSuccess) e = column_runs(nullptr, d_off, d_runs);
      if (e == hipSuccess) {
        runs.resize(4 * (size_t)total);
        e = hipMemcpy(runs.data(), d_runs, sizeof(int64_t) * 4 * (size_t)total, hipMemcpyDeviceToHost);
      }
    }
    (void)hipFree(d_cnt);
    (void)hipFree(d_off);
    (void)hipFree(d_runs);
    if (e != hipSuccess) return hip_fail(e, "post-selection");
    if (total == 0) return fail(GPE_ERR_ARG, "geometry: the active set is empty");
  }
  Layout lay;
  std::string err = layout_from_runs(geom->n, (int64_t)(runs.size() / 4), runs.data(), lay);
  if (!err.empty()) return fail(GPE_ERR_ARG, "%s", err.c_str());
  return finish_grid(geom, std::move(lay), device, out);
}

gpe_status gpe_remap(gpe_grid src, gpe_grid dst, gpe_dtype dtype, const void* psi_src, void* psi_dst, void* stream) {
  gpe_status st = check_grid(src);
  if (st == GPE_OK) st = check_grid(dst);
  if (st == GPE_OK) st = check_dtype(dtype);
  if (st == GPE_OK) st = check_ptr(psi_src, "psi_src");
  if (st == GPE_OK) st = check_ptr(psi_dst, "psi_dst");
  if (st != GPE_OK) return st;
  if (src->device != dst->device) return fail(GPE_ERR_ARG, "source and destination grids are on different devices");
  for (int d = 0; d < 3; ++d)
    if (src->lay.n[d] != dst->lay.n[d]) return fail(GPE_ERR_ARG, "source and destination grids have different boxes");
  if (psi_src == psi_dst) return fail(GPE_ERR_ARG, "psi_src and psi_dst must not be the same buffer");
  // intervals of the destination array: copied from consecutive source sites or zero
  const Layout& A = src->lay;
  const Layout& B = dst->lay;
  std::vector<int64_t> ivd, ivs;
  auto emit = [&](int64_t d0, int64_t s0) {
    if (!ivd.empty() && ((s0 < 0 && ivs.back() < 0) ||
                         (s0 >= 0 && ivs.back() >= 0 && ivs.back() + (d0 - ivd.back()) == s0)))
      return;   // continues the previous interval
    ivd.push_back(d0);
    ivs.push_back(s0);
  };
  int64_t q = 0;
  const int64_t na = A.n_runs();
  for (int64_t r = 0; r < B.n_runs(); ++r) {
    const int64_t i = B.run_i[r], j = B.run_j[r], k0 = B.run_k0[r], k1 = B.run_k1[r], d0 = B.run_start[r];
    auto before = [&](int64_t x) {   // source run x lies wholly before this destination run
      return A.run_i[x] < i || (A.run_i[x] == i && (A.run_j[x] < j || (A.run_j[x] == j && A.run_k1[x] <= k0)));
    };
    while (q < na && before(q)) ++q;
    int64_t cur = k0;
    for (int64_t x = q; x < na && A.run_i[x] == i && A.run_j[x] == j && A.run_k0[x] < k1; ++x) {
      const int64_t o0 = std::max(k0, A.run_k0[x]), o1 = std::min(k1, A.run_k1[x]);
      if (o0 > cur) emit(d0 + (cur - k0), -1);
      if (o0 < o1) emit(d0 + (o0 - k0), A.run_start[x] + (o0 - A.run_k0[x]));
      cur = std::max(cur, o1);
    }
    if (cur < k1) emit(d0 + (cur - k0), -1);
  }
  DeviceGuard dg(dst->device);
  hipStream_t s = (hipStream_t)stream;
  int64_t* d_iv = nullptr;
  const int64_t n_iv = (int64_t)ivd.size();
  HIP_TRY(hipMalloc((void**)&d_iv, sizeof(int64_t) * 2 * n_iv));
  hipError_t e = hipMemcpy(d_iv, ivd.data(), sizeof(int64_t) * n_iv, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d_iv + n_iv, ivs.data(), sizeof(int64_t) * n_iv, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = dtype == GPE_C128 ? run_remap<double>(d_iv, d_iv + n_iv, n_iv, B.n_active, psi_src, psi_dst, s)
                          : run_remap<float>(d_iv, d_iv + n_iv, n_iv, B.n_active, psi_src, psi_dst, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(d_iv);
  if (e != hipSuccess) return hip_fail(e, "remap");
  return GPE_OK;
}

gpe_status gpe_grid_set_stencil(gpe_grid g, int32_t points) {
  if (!g) return fail(GPE_ERR_ARG, "grid is NULL");
  if (points != 7 && points != 19 && points != 27) return fail(GPE_ERR_ARG, "stencil must have 7, 19 or 27 points");
  if (points == 27) {
    const double* h = g->lay.h;
    const double hm = std::max(h[0], std::max(h[1], h[2])), hn = std::min(h[0], std::min(h[1], h[2]));
    if (hm - hn > 1e-12 * hm) return fail(GPE_ERR_ARG, "the 27-point stencil needs equal spacings");
  }
  if (points == 19) build_hoc_segments(g->lay);
  if (points == 27) build_c27_segments(g->lay);
  if (g->device >= 0 && g->prob) {
    if (points != 7) {
      DeviceGuard dg(g->device);
      gpe_status st = g->prob->enable_hoc(g->lay, points);
      if (st != GPE_OK) return st;
    }
    g->prob->stencil = points;
    DeviceGuard dg(g->device);
    gpe_status st = prepare_tables(g->prob.get());
    if (st != GPE_OK) return st;
  }
  g->stencil = points;
  return GPE_OK;
}

gpe_status gpe_grid_get_stencil(gpe_grid g, int32_t* points) {
  if (!g || !points) return fail(GPE_ERR_ARG, "grid or points is NULL");
  *points = g->stencil;
  return GPE_OK;
}

gpe_status gpe_grid_stencil_segments(gpe_grid g, int32_t points, int64_t* n_segments, int32_t* out_host) {
  if (!g || !n_segments) return fail(GPE_ERR_ARG, "grid or n_segments is NULL");
  if (points != 19 && points != 27) return fail(GPE_ERR_ARG, "tap tables exist for 19 and 27 points");
  const bool c27 = points == 27;
  if (c27) build_c27_segments(g->lay); else build_hoc_segments(g->lay);
  const std::vector<SegHead>& hh = c27 ? g->lay.c27_heads : g->lay.hoc_heads;
  const int ntaps = c27 ? C27_TAPS : HOC_TAPS;
  const int64_t n = (int64_t)hh.size() - 1;
  *n_segments = n;
  if (!out_host) return GPE_OK;
  for (int64_t q = 0; q < n; ++q) {
    int32_t* o = out_host + (4 + ntaps) * q;
    o[0] = hh[q].start;
    o[1] = hh[q + 1].start - hh[q].start;
    o[2] = hh[q].flags;
    for (int t = 0; t < ntaps; ++t) o[3 + t] = c27 ? g->lay.c27_nbs[q].off[t] : g->lay.hoc_nbs[q].off[t];
    o[3 + ntaps] = 0;
  }
  return GPE_OK;
}

gpe_status gpe_grid_info(gpe_grid g, int64_t* n_active, int64_t* n_runs, int64_t* n_segments) {
  if (!g) return fail(GPE_ERR_ARG, "grid is NULL");
  if (n_active) *n_active = g->lay.n_active;
  if (n_runs) *n_runs = g->lay.n_runs();
  if (n_segments) *n_segments = g->lay.n_segments();
  return GPE_OK;
}

gpe_status gpe_grid_segments(gpe_grid g, int32_t* out) {
  if (!g || !out) return fail(GPE_ERR_ARG, "grid or out is NULL");
  const Layout& L = g->lay;
  for (int64_t q = 0; q < L.n_segments(); ++q) {
    int32_t* o = out + 8 * q;
    o[0] = L.heads[q].start;
    o[1] = L.heads[q + 1].start - L.heads[q].start;
    o[2] = L.heads[q].flags;
    o[3] = L.nbs[q].xm;
    o[4] = L.nbs[q].xp;
    o[5] = L.nbs[q].ym;
    o[6] = L.nbs[q].yp;
    o[7] = 0;
  }
  return GPE_OK;
}

gpe_status gpe_grid_runs(gpe_grid g, int64_t* out) {
  if (!g || !out) return fail(GPE_ERR_ARG, "grid or out is NULL");
  const Layout& L = g->lay;
  for (int64_t r = 0; r < L.n_runs(); ++r) {
    out[5 * r] = L.run_i[r];
    out[5 * r + 1] = L.run_j[r];
    out[5 * r + 2] = L.run_k0[r];
    out[5 * r + 3] = L.run_k1[r];
    out[5 * r + 4] = L.run_start[r];
  }
  return GPE_OK;
}

gpe_status gpe_grid_destroy(gpe_grid g) {
  delete g;
  return GPE_OK;
}

gpe_status gpe_work_bytes(gpe_grid g, gpe_dtype dtype, int32_t mode, int64_t nsteps, int64_t ckpt_every,
                          size_t* bytes) {
  if (!g || !bytes) return fail(GPE_ERR_ARG, "grid or bytes is NULL");
  gpe_status st = check_dtype(dtype);
  if (st != GPE_OK) return st;
  if (mode < GPE_MODE_ITP || mode > GPE_MODE_ITP_REAL) return fail(GPE_ERR_ARG, "unknown mode");
  if (nsteps < 0 || ckpt_every < 0) return fail(GPE_ERR_ARG, "nsteps and ckpt_every must be >= 0");
  *bytes = work_bytes_for(g->lay.n_active, dtype, mode, nsteps, ckpt_every);
  return GPE_OK;
}

gpe_status gpe_pack(gpe_grid g, gpe_dtype dtype, const void* box_dev, void* compact_dev, void* stream) {
  gpe_status st = check_grid(g);
  if (st == GPE_OK) st = check_dtype(dtype);
  if (st == GPE_OK) st = check_ptr(box_dev, "box");
  if (st == GPE_OK) st = check_ptr(compact_dev, "compact");
  if (st != GPE_OK) return st;
  DeviceGuard dg(g->device);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = dtype == GPE_C128
                     ? run_pack<double>(g->d_run_base, g->d_run_start, g->lay.n_runs(), g->lay.n_active, box_dev,
                                        compact_dev, false, s)
                     : run_pack<float>(g->d_run_base, g->d_run_start, g->lay.n_runs(), g->lay.n_active, box_dev,
                                       compact_dev, false, s);
  if (e != hipSuccess) return hip_fail(e, "pack");
  return GPE_OK;
}

gpe_status gpe_pack_real(gpe_grid g, gpe_dtype dtype, const void* box_dev, void* compact_dev, void* stream) {
  gpe_status st = check_grid(g);
  if (st == GPE_OK) st = check_dtype(dtype);
  if (st == GPE_OK) st = check_ptr(box_dev, "box");
  if (st == GPE_OK) st = check_ptr(compact_dev, "compact");
  if (st != GPE_OK) return st;
  DeviceGuard dg(g->device);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = dtype == GPE_C128
                     ? run_pack<double>(g->d_run_base, g->d_run_start, g->lay.n_runs(), g->lay.n_active, box_dev,
                                        compact_dev, false, s, true)
                     : run_pack<float>(g->d_run_base, g->d_run_start, g->lay.n_runs(), g->lay.n_active, box_dev,
                                       compact_dev, false, s, true);
  if (e != hipSuccess) return hip_fail(e, "pack_real");
  return GPE_OK;
}

gpe_status gpe_unpack(gpe_grid g, gpe_dtype dtype, const void* compact_dev, void* box_dev, void* stream) {
  gpe_status st = check_grid(g);
  if (st == GPE_OK) st = check_dtype(dtype);
  if (st == GPE_OK) st = check_ptr(box_dev, "box");
  if (st == GPE_OK) st = check_ptr(compact_dev, "compact");
  if (st != GPE_OK) return st;
  DeviceGuard dg(g->device);
  hipStream_t s = (hipStream_t)stream;
  const int64_t nbox = g->lay.n[0] * g->lay.n[1] * g->lay.n[2];
  hipError_t e = dtype == GPE_C128 ? run_fill_zero<double>(box_dev, nbox, s) : run_fill_zero<float>(box_dev, nbox, s);
  if (e == hipSuccess)
    e = dtype == GPE_C128 ? run_pack<double>(g->d_run_base, g->d_run_start, g->lay.n_runs(), g->lay.n_active,
                                             compact_dev, box_dev, true, s)
                          : run_pack<float>(g->d_run_base, g->d_run_start, g->lay.n_runs(), g->lay.n_active,
                                            compact_dev, box_dev, true, s);
  if (e != hipSuccess) return hip_fail(e, "unpack");
  return GPE_OK;
}

static gpe_status check_work(const void* work, size_t have, size_t need) {
  if (need > 0) {
    gpe_status st = check_ptr(work, "work");
    if (st != GPE_OK) return st;
  }
  if (have < need) return fail(GPE_ERR_ARG, "work buffer too small: %zu bytes given, %zu needed", have, need);
  return GPE_OK;
}

static gpe_status imag_time_impl(gpe_grid g, gpe_dtype dtype, void* psi, const gpe_potential* pot,
                                 const gpe_params* prm, int64_t nsteps, void* work, size_t work_bytes, void* stream,
                                 gpe_obs* final_host, gpe_obs* history_dev, bool real) {
  gpe_status st = check_grid(g);
  if (st == GPE_OK) st = check_dtype(dtype);
  if (st == GPE_OK) st = check_ptr(psi, "psi");
  if (st == GPE_OK) st = check_pot(pot);
  if (st == GPE_OK) st = check_params(prm);
  if (st != GPE_OK) return st;
  if (prm->integrator != GPE_RK4) return fail(GPE_ERR_ARG, "params.integrator must be 0 for imaginary time");
  if (nsteps < 0) return fail(GPE_ERR_ARG, "nsteps must be >= 0");
  if (prm->obs_every > 0 && !history_dev) return fail(GPE_ERR_ARG, "obs_every > 0 needs history_dev");
  st = check_work(work, work_bytes,
                  work_bytes_for(g->lay.n_active, dtype, real ? GPE_MODE_ITP_REAL : GPE_MODE_ITP, nsteps, 0));
  if (st != GPE_OK) return st;
  DeviceGuard dg(g->device);
  hipStream_t s = (hipStream_t)stream;
  Ctx c;
  st = make_ctx(g->prob.get(), g->prob->config, s, c);
  if (st != GPE_OK) return st;
  Ordered ord(g->prob.get(), s);
  if (ord.st != GPE_OK) return ord.st;
  std::vector<InstParams> ps{make_params(pot, prm, 0.0)};
  st = g->prob->upload(*c.cs, ps, s);
  if (st != GPE_OK) return st;
  if (!prm->skip_stability_check) {
    st = dtype == GPE_C128 ? itp_stability<double>(c, ps.data(), pot->field, psi, real)
                           : itp_stability<float>(c, ps.data(), pot->field, psi, real);
    if (st != GPE_OK) return st;
  }
  st = dtype == GPE_C128 ? drive_itp<double>(c, psi, pot->field, nsteps, work, prm->obs_every, history_dev, real)
                         : drive_itp<float>(c, psi, pot->field, nsteps, work, prm->obs_every, history_dev, real);
  if (st != GPE_OK) return st;
  if (final_host) {
    st = dtype == GPE_C128 ? drive_observe<double>(c, psi, pot->field, false, 0, real)
                           : drive_observe<float>(c, psi, pot->field, false, 0, real);
    if (st != GPE_OK) return st;
    return read_obs(*g->prob, final_host, s);
  }
  return GPE_OK;
}

gpe_status gpe_imag_time(gpe_grid g, gpe_dtype dtype, void* psi, const gpe_potential* pot, const gpe_params* prm,
                         int64_t nsteps, void* work, size_t work_bytes, void* stream, gpe_obs* final_host,
                         gpe_obs* history_dev) {
  return imag_time_impl(g, dtype, psi, pot, prm, nsteps, work, work_bytes, stream, final_host, history_dev, false);
}

gpe_status gpe_imag_time_real(gpe_grid g, gpe_dtype dtype, void* psi, const gpe_potential* pot,
                              const gpe_params* prm, int64_t nsteps, void* work, size_t work_bytes, void* stream,
                              gpe_obs* final_host, gpe_obs* history_dev) {
  return imag_time_impl(g, dtype, psi, pot, prm, nsteps, work, work_bytes, stream, final_host, history_dev, true);
}

gpe_status gpe_real_time(gpe_grid g, gpe_dtype dtype, void* psi, const gpe_potential* pot, const gpe_params* prm,
                         double t0, int64_t nsteps, void* work, size_t work_bytes, void* stream, gpe_obs* final_host,
                         gpe_obs* history_dev) {
  gpe_status st = check_grid(g);
  if (st == GPE_OK) st = check_dtype(dtype);
  if (st == GPE_OK) st = check_ptr(psi, "psi");
  if (st == GPE_OK) st = check_pot(pot);
  if (st == GPE_OK) st = check_params(prm);
  if (st != GPE_OK) return st;
  if (!std::isfinite(t0)) return fail(GPE_ERR_ARG, "t0 must be finite");
  if (nsteps < 0) return fail(GPE_ERR_ARG, "nsteps must be >= 0");
  if (prm->obs_every > 0 && !history_dev) return fail(GPE_ERR_ARG, "obs_every > 0 needs history_dev");
  st = check_work(work, work_bytes,
                  work_bytes_for(g->lay.n_active, dtype, rt_work_mode(prm->integrator), nsteps, 0));
  if (st != GPE_OK) return st;
  DeviceGuard dg(g->device);
  hipStream_t s = (hipStream_t)stream;
  Ctx c;
  st = make_ctx(g->prob.get(), g->prob->config, s, c);
  if (st != GPE_OK) return st;
  Ordered ord(g->prob.get(), s);
  if (ord.st != GPE_OK) return ord.st;
  std::vector<InstParams> ps{make_params(pot, prm, t0)};
  st = g->prob->upload(*c.cs, ps, s);
  if (st != GPE_OK) return st;
  if (!prm->skip_stability_check) {
    st = dtype == GPE_C128 ? rt_stability<double>(c, ps.data(), pot->field, psi, prm->integrator)
                           : rt_stability<float>(c, ps.data(), pot->field, psi, prm->integrator);
    if (st != GPE_OK) return st;
  }
  st = dtype == GPE_C128
           ? drive_rt<double>(c, psi, pot->field, nsteps, work, prm->obs_every, history_dev, prm->integrator)
           : drive_rt<float>(c, psi, pot->field, nsteps, work, prm->obs_every, history_dev, prm->integrator);
  if (st != GPE_OK) return st;
  if (final_host) {
    // observation at the final time t0 + nsteps dt
    st = dtype == GPE_C128 ? drive_observe<double>(c, psi, pot->field, false, nsteps)
                           : drive_observe<float>(c, psi, pot->field, false, nsteps);
    if (st != GPE_OK) return st;
    return read_obs(*g->prob, final_host, s);
  }
  return GPE_OK;
}

}  // extern "C"

// ---- real time without allocation -------------------------------------------
// The stage states of gpe_real_time_noalloc live in this file-scope device
// array: every GPU the library runs on holds its own copy from module load
// until the process ends.  In host code `scratch` names a host-side stand-in,
// so kernels are given the device address that hipGetSymbolAddress returns,
// looked up once per device with that device current.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// device address of `scratch` on `device` (which must be current)
gpe_status scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return fail(GPE_ERR_ARG, "device %d out of range", device);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(GPE_ERR_DEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_dev[device] = p;
  }
  *out = g_scratch_dev[device];
  return GPE_OK;
}
}  // namespace

extern "C" {

size_t gpe_noalloc_scratch_bytes(void) { return kNoAllocScratchBytes; }

gpe_status gpe_real_time_noalloc(gpe_grid g, gpe_dtype dtype, void* psi, const gpe_potential* pot,
                                 const gpe_params* prm, double t0, int64_t nsteps, void* stream,
                                 gpe_obs* final_host, gpe_obs* history_dev) {
  gpe_status st = check_grid(g);
  if (st == GPE_OK) st = check_dtype(dtype);
  if (st == GPE_OK) st = check_ptr(psi, "psi");
  if (st == GPE_OK) st = check_pot(pot);
  if (st == GPE_OK) st = check_params(prm);
  if (st != GPE_OK) return st;
  if (!std::isfinite(t0)) return fail(GPE_ERR_ARG, "t0 must be finite");
  if (nsteps < 0) return fail(GPE_ERR_ARG, "nsteps must be >= 0");
  if (prm->obs_every > 0 && !history_dev) return fail(GPE_ERR_ARG, "obs_every > 0 needs history_dev");
  const size_t need = work_bytes_for(g->lay.n_active, dtype, rt_work_mode(prm->integrator), nsteps, 0);
  if (need > kNoAllocScratchBytes)
    return fail(GPE_ERR_ARG, "the stage states need %zu bytes; the allocation-free call holds at most %zu", need,
                kNoAllocScratchBytes);
  DeviceGuard dg(g->device);
  if (!dg.ok) return fail(GPE_ERR_DEVICE, "hipSetDevice(%d) failed", g->device);
  void* work = nullptr;
  st = scratch_address(g->device, &work);
  if (st != GPE_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  Ctx c;
  // the launch tables exist since the grid was created or its variant chosen
  st = make_ctx(g->prob.get(), g->prob->config, s, c, false);
  if (st != GPE_OK) return st;
  Ordered ord(g->prob.get(), s);
  if (ord.st != GPE_OK) return ord.st;
  const InstParams ip = make_params(pot, prm, t0);
  st = g->prob->upload(*c.cs, &ip, s);
  if (st != GPE_OK) return st;
  if (!prm->skip_stability_check) {
    st = dtype == GPE_C128 ? rt_stability<double>(c, &ip, pot->field, psi, prm->integrator)
                           : rt_stability<float>(c, &ip, pot->field, psi, prm->integrator);
    if (st != GPE_OK) return st;
  }
  st = dtype == GPE_C128
           ? drive_rt<double>(c, psi, pot->field, nsteps, work, prm->obs_every, history_dev, prm->integrator)
           : drive_rt<float>(c, psi, pot->field, nsteps, work, prm->obs_every, history_dev, prm->integrator);
  if (st != GPE_OK) return st;
  if (final_host) {
    st = dtype == GPE_C128 ? drive_observe<double>(c, psi, pot->field, false, nsteps)
                           : drive_observe<float>(c, psi, pot->field, false, nsteps);
    if (st != GPE_OK) return st;
    return read_obs(*g->prob, final_host, s);
  }
  return GPE_OK;
}

gpe_status gpe_observe(gpe_grid g, gpe_dtype dtype, const void* psi, const gpe_potential* pot, double t, double gg,
                       void* stream, gpe_obs* out_host) {
  gpe_status st = check_grid(g);
  if (st == GPE_OK) st = check_dtype(dtype);
  if (st == GPE_OK) st = check_ptr(psi, "psi");
  if (st == GPE_OK) st = check_pot(pot);
  if (st != GPE_OK) return st;
  if (!out_host) return fail(GPE_ERR_ARG, "out_host is NULL");
  if (!std::isfinite(t) || !std::isfinite(gg)) return fail(GPE_ERR_ARG, "t and g must be finite");
  DeviceGuard dg(g->device);
  hipStream_t s = (hipStream_t)stream;
  Ctx c;
  st = make_ctx(g->prob.get(), g->prob->config, s, c);
  if (st != GPE_OK) return st;
  gpe_params prm;
  std::memset(&prm, 0, sizeof prm);
  prm.g = gg;
  prm.dt = 1.0;
  Ordered ord(g->prob.get(), s);
  if (ord.st != GPE_OK) return ord.st;
  std::vector<InstParams> ps{make_params(pot, &prm, t)};
  st = g->prob->upload(*c.cs, ps, s);
  if (st != GPE_OK) return st;
  st = dtype == GPE_C128 ? drive_observe<double>(c, psi, pot->field, false, 0)
                         : drive_observe<float>(c, psi, pot->field, false, 0);
  if (st != GPE_OK) return st;
  return read_obs(*g->prob, out_host, s);
}

gpe_status gpe_overlap(gpe_grid g, gpe_dtype dtype, const void* a, const void* b, void* stream, double* out_host) {
  gpe_status st = check_grid(g);
  if (st == GPE_OK) st = check_dtype(dtype);
  if (st == GPE_OK) st = check_ptr(a, "a");
  if (st == GPE_OK) st = check_ptr(b, "b");
  if (st != GPE_OK) return st;
  if (!out_host) return fail(GPE_ERR_ARG, "out_host is NULL");
  DeviceGuard dg(g->device);
  hipStream_t s = (hipStream_t)stream;
  Ctx c;
  st = make_ctx(g->prob.get(), g->prob->config, s, c);
  if (st != GPE_OK) return st;
  Ordered ord(g->prob.get(), s);
  if (ord.st != GPE_OK) return ord.st;
  std::vector<InstParams> ps{make_params(nullptr, nullptr, 0.0)};
  st = g->prob->upload(*c.cs, ps, s);
  if (st != GPE_OK) return st;
  hipError_t e = dtype == GPE_C128 ? run_overlap<double>(c.pl, c.cfg, a, b, s) : run_overlap<float>(c.pl, c.cfg, a, b, s);
  if (e == hipSuccess) e = run_finalize(c.pl, FIN_OVERLAP, nullptr, s);
  if (e != hipSuccess) return hip_fail(e, "overlap");
  InstOut o;
  HIP_TRY(hipMemcpyAsync(&o, g->prob->d_out, sizeof(InstOut), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  out_host[0] = o.ov_re;
  out_host[1] = o.ov_im;
  return GPE_OK;
}

gpe_status gpe_fidelity_grad(gpe_grid g, gpe_dtype dtype, const void* psi0, const void* psi_target,
                             const gpe_potential* pot, const gpe_params* prm, double t0, int64_t nsteps,
                             int64_t ckpt_every, void* work, size_t work_bytes, void* stream, double* loss_host,
                             double* grad_host, void* psi_final) {
  gpe_status st = check_grid(g);
  if (st == GPE_OK) st = check_dtype(dtype);
  if (st == GPE_OK) st = check_ptr(psi0, "psi0");
  if (st == GPE_OK) st = check_ptr(psi_target, "psi_target");
  if (st == GPE_OK) st = check_pot(pot);
  if (st == GPE_OK) st = check_params(prm);
  if (st != GPE_OK) return st;
  if (pot->kind != GPE_POT_RF_RAMP && pot->kind != GPE_POT_SHELL_RAMP)
    return fail(GPE_ERR_ARG, "the fidelity gradient needs a ramped potential (RF_RAMP or SHELL_RAMP)");
  if (prm->integrator != GPE_RK4) return fail(GPE_ERR_ARG, "the fidelity gradient is the adjoint of RK4 only");
  if (!loss_host || !grad_host) return fail(GPE_ERR_ARG, "loss_host and grad_host are required");
  if (psi_final) {
    st = check_ptr(psi_final, "psi_final");
    if (st != GPE_OK) return st;
  }
  if (nsteps < 1 || ckpt_every < 0) return fail(GPE_ERR_ARG, "nsteps must be >= 1 and ckpt_every >= 0");
  if (!std::isfinite(t0)) return fail(GPE_ERR_ARG, "t0 must be finite");
  st = check_work(work, work_bytes, work_bytes_for(g->lay.n_active, dtype, GPE_MODE_ADJ, nsteps, ckpt_every));
  if (st != GPE_OK) return st;
  DeviceGuard dg(g->device);
  hipStream_t s = (hipStream_t)stream;
  Ctx c;
  st = make_ctx(g->prob.get(), g->prob->config, s, c);
  if (st != GPE_OK) return st;
  Ordered ord(g->prob.get(), s);
  if (ord.st != GPE_OK) return ord.st;
  std::vector<InstParams> ps{make_params(pot, prm, t0)};
  st = g->prob->upload(*c.cs, ps, s);
  if (st != GPE_OK) return st;
  if (!prm->skip_stability_check) {
    st = dtype == GPE_C128 ? rt_stability<double>(c, ps.data(), pot->field, psi0, GPE_RK4, 3.0)
                           : rt_stability<float>(c, ps.data(), pot->field, psi0, GPE_RK4, 3.0);
    if (st != GPE_OK) return st;
  }
  st = dtype == GPE_C128 ? drive_adjoint<double>(c, psi0, psi_target, pot->field, nsteps, ckpt_every, work, psi_final)
                         : drive_adjoint<float>(c, psi0, psi_target, pot->field, nsteps, ckpt_every, work, psi_final);
  if (st != GPE_OK) return st;
  HIP_TRY(hipStreamSynchronize(s));
  return read_loss_grad(*g->prob, loss_host, grad_host, pot->n_knots);
}

// ---- staged ramps (Sec. V) --------------------------------------------------

gpe_status gpe_staged_ramp_grids(const gpe_geometry* geom, gpe_dtype dtype, int32_t n_fields,
                                 const void* const* fields_box, const double* mus_host, double cutoff_factor,
                                 int device, gpe_grid* grids_out, double* cutoffs_host) {
  if (!grids_out) return fail(GPE_ERR_ARG, "grids_out is NULL");
  if (n_fields < 2) return fail(GPE_ERR_ARG, "a staged ramp needs at least two stage potentials");
  for (int32_t i = 0; i + 1 < n_fields; ++i) grids_out[i] = nullptr;
  if (!fields_box || !mus_host) return fail(GPE_ERR_ARG, "fields_box and mus_host are required");
  for (int32_t i = 0; i < n_fields; ++i)
    if (!std::isfinite(mus_host[i])) return fail(GPE_ERR_ARG, "mu %d is not finite", i);
  if (std::isnan(cutoff_factor)) return fail(GPE_ERR_ARG, "cutoff_factor is NaN");
  // Sec. V: the grid of stage i keeps the points below 5 max(mu_i, mu_{i+1})
  const double f = cutoff_factor > 0.0 ? cutoff_factor : 5.0;
  for (int32_t i = 0; i + 1 < n_fields; ++i) {
    const double cut = f * std::max(mus_host[i], mus_host[i + 1]);
    if (cutoffs_host) cutoffs_host[i] = cut;
    gpe_status st = gpe_grid_create_threshold(geom, dtype, fields_box[i], fields_box[i + 1], cut, device,
                                              &grids_out[i]);
    if (st != GPE_OK) {
      const std::string msg = t_err;
      for (int32_t j = 0; j < i; ++j) {
        (void)gpe_grid_destroy(grids_out[j]);
        grids_out[j] = nullptr;
      }
      return fail(st, "stage %d: %s", i, msg.c_str());
    }
  }
  return GPE_OK;
}

static bool same_layout(const Layout& a, const Layout& b) {
  return a.n_active == b.n_active && a.run_i == b.run_i && a.run_j == b.run_j && a.run_k0 == b.run_k0 &&
         a.run_k1 == b.run_k1;
}

static size_t staged_stage_bytes(int64_t n, int dtype, int integrator) {
  Carver c(nullptr);
  c.take((size_t)n * rsize(dtype));
  c.take((size_t)n * rsize(dtype));
  c.take(work_bytes_for(n, dtype, rt_work_mode(integrator), 0, 0));
  return c.off;
}

gpe_status gpe_staged_ramp_work_bytes(int32_t n_stages, const gpe_grid* grids, gpe_dtype dtype, int32_t integrator,
                                      size_t* bytes) {
  if (!grids || !bytes || n_stages < 1) return fail(GPE_ERR_ARG, "need n_stages >= 1 grids and bytes");
  gpe_status st = check_dtype(dtype);
  if (st != GPE_OK) return st;
  if (integrator != GPE_RK4 && integrator != GPE_RKHE3 && integrator != GPE_RKCK)
    return fail(GPE_ERR_ARG, "unknown integrator");
  size_t m = 0;
  for (int32_t i = 0; i < n_stages; ++i) {
    if (!grids[i]) return fail(GPE_ERR_ARG, "grid %d is NULL", i);
    m = std::max(m, staged_stage_bytes(grids[i]->lay.n_active, dtype, integrator));
  }
  *bytes = m;
  return GPE_OK;
}

gpe_status gpe_staged_ramp_run(gpe_grid src, const void* psi_src, int32_t n_stages, const gpe_grid* grids,
                               void* const* psi_stage, gpe_dtype dtype, const void* const* fields_box,
                               const gpe_params* prm, double t0, int64_t steps_per_stage, void* work,
                               size_t work_bytes, void* stream, double* records_host) {
  gpe_status st = check_grid(src);
  if (st == GPE_OK) st = check_dtype(dtype);
  if (st == GPE_OK) st = check_ptr(psi_src, "psi_src");
  if (st == GPE_OK) st = check_params(prm);
  if (st != GPE_OK) return st;
  if (n_stages < 1 || !grids || !psi_stage || !fields_box || !records_host)
    return fail(GPE_ERR_ARG, "need n_stages >= 1, grids, psi_stage, fields_box and records_host");
  if (steps_per_stage < 1 || !std::isfinite(t0)) return fail(GPE_ERR_ARG, "steps_per_stage must be >= 1, t0 finite");
  for (int32_t i = 0; i < n_stages; ++i) {
    st = check_grid(grids[i]);
    if (st == GPE_OK) st = check_ptr(psi_stage[i], "psi_stage");
    if (st == GPE_OK) st = check_ptr(fields_box[i], "fields_box");
    if (st != GPE_OK) return st;
    if (grids[i]->device != src->device) return fail(GPE_ERR_ARG, "stage %d: grids on different devices", i);
    for (int d = 0; d < 3; ++d)
      if (grids[i]->lay.n[d] != src->lay.n[d]) return fail(GPE_ERR_ARG, "stage %d: a different box", i);
    const void* prev = i == 0 ? psi_src : psi_stage[i - 1];
    if (psi_stage[i] == prev) return fail(GPE_ERR_ARG, "stage %d: psi buffer aliases the previous one", i);
  }
  st = check_ptr(fields_box[n_stages], "fields_box");
  if (st != GPE_OK) return st;
  size_t need = 0;
  st = gpe_staged_ramp_work_bytes(n_stages, grids, dtype, prm->integrator, &need);
  if (st != GPE_OK) return st;
  st = check_work(work, work_bytes, need);
  if (st != GPE_OK) return st;
  const double dt = prm->dt;
  const size_t csz = csize(dtype);
  for (int32_t i = 0; i < n_stages; ++i) {
    gpe_grid g = grids[i];
    const gpe_grid prev = i == 0 ? src : grids[i - 1];
    const void* psi_prev = i == 0 ? psi_src : psi_stage[i - 1];
    // carry psi over to the stage's grid (an unchanged selection is a plain copy)
    if (same_layout(prev->lay, g->lay)) {
      DeviceGuard dg(g->device);
      HIP_TRY(hipMemcpyAsync(psi_stage[i], psi_prev, (size_t)g->lay.n_active * csz, hipMemcpyDeviceToDevice,
                             (hipStream_t)stream));
    } else {
      st = gpe_remap(prev, g, dtype, psi_prev, psi_stage[i], stream);
      if (st != GPE_OK) return st;
    }
    // the two stage potentials on the stage's grid, then the stage's steps with
    // V interpolated linearly in time from V_i at t_i to V_{i+1} at t_{i+1}
    Carver cv(work);
    void* va = cv.take((size_t)g->lay.n_active * rsize(dtype));
    void* vb = cv.take((size_t)g->lay.n_active * rsize(dtype));
    void* rt_work = cv.take(work_bytes_for(g->lay.n_active, dtype, rt_work_mode(prm->integrator), 0, 0));
    st = gpe_pack_real(g, dtype, fields_box[i], va, stream);
    if (st == GPE_OK) st = gpe_pack_real(g, dtype, fields_box[i + 1], vb, stream);
    if (st != GPE_OK) return st;
    const double ta = t0 + (double)i * (double)steps_per_stage * dt;
    const double tb = ta + (double)steps_per_stage * dt;
    const double kt[2] = {ta, tb};
    gpe_potential pot;
    std::memset(&pot, 0, sizeof pot);
    pot.kind = GPE_POT_LERP;
    pot.n_knots = 2;
    pot.field = va;
    pot.field2 = vb;
    pot.knot_t = kt;
    gpe_obs kept, end;
    st = gpe_observe(g, dtype, psi_stage[i], &pot, ta, prm->g, stream, &kept);
    if (st != GPE_OK) return st;
    gpe_params p = *prm;
    p.obs_every = 0;
    st = gpe_real_time(g, dtype, psi_stage[i], &pot, &p, ta, steps_per_stage, rt_work,
                       work_bytes - (size_t)((char*)rt_work - (char*)work), stream, &end, nullptr);
    if (st != GPE_OK) return fail(st, "stage %d: %s", i, std::string(t_err).c_str());
    double* r = records_host + 4 * (size_t)i;
    r[0] = kept.norm;
    r[1] = end.norm;
    r[2] = end.energy;
    r[3] = end.mu;
  }
  return GPE_OK;
}

// ---- batches --------------------------------------------------------------

gpe_status gpe_batch_create(int32_t n, const gpe_grid* grids, int device, gpe_batch* out) {
  if (!out) return fail(GPE_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (n < 1 || !grids) return fail(GPE_ERR_ARG, "need at least one grid");
  if (device < 0) return fail(GPE_ERR_ARG, "batch needs a device");
  std::vector<const Layout*> lays;
  for (int i = 0; i < n; ++i) {
    if (!grids[i]) return fail(GPE_ERR_ARG, "grid %d is NULL", i);
    lays.push_back(&grids[i]->lay);
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device >= ndev) return fail(GPE_ERR_DEVICE, "device %d not available", device);
  gpe_batch b = new (std::nothrow) gpe_batch_s();
  if (!b) return fail(GPE_ERR_ALLOC, "out of host memory");
  b->grids.assign(grids, grids + n);
  b->device = device;
  b->prob.reset(new (std::nothrow) Problem());
  if (!b->prob) {
    delete b;
    return fail(GPE_ERR_ALLOC, "out of host memory");
  }
  gpe_status st = b->prob->build(device, lays);
  if (st == GPE_OK) {
    DeviceGuard dg(device);
    st = prepare_tables(b->prob.get());
  }
  if (st != GPE_OK) {
    delete b;
    return st;
  }
  *out = b;
  return GPE_OK;
}

gpe_status gpe_batch_offsets(gpe_batch b, int64_t* offsets) {
  if (!b || !offsets) return fail(GPE_ERR_ARG, "batch or offsets is NULL");
  for (int i = 0; i <= b->prob->n_inst; ++i) offsets[i] = b->prob->inst_site[i];
  return GPE_OK;
}

gpe_status gpe_batch_destroy(gpe_batch b) {
  delete b;
  return GPE_OK;
}

gpe_status gpe_batch_work_bytes(gpe_batch b, gpe_dtype dtype, int32_t mode, int64_t nsteps, int64_t ckpt_every,
                                size_t* bytes) {
  if (!b || !bytes) return fail(GPE_ERR_ARG, "batch or bytes is NULL");
  gpe_status st = check_dtype(dtype);
  if (st != GPE_OK) return st;
  if (mode < GPE_MODE_ITP || mode > GPE_MODE_ITP_REAL) return fail(GPE_ERR_ARG, "unknown mode");
  if (nsteps < 0 || ckpt_every < 0) return fail(GPE_ERR_ARG, "nsteps and ckpt_every must be >= 0");
  *bytes = work_bytes_for(b->prob->total, dtype, mode, nsteps, ckpt_every);
  return GPE_OK;
}

static gpe_status batch_params(gpe_batch b, const gpe_ramp* ramps, const gpe_params* prms, double t0,
                               std::vector<InstParams>& ps) {
  if (!ramps || !prms) return fail(GPE_ERR_ARG, "ramps and params are required");
  const int n = b->prob->n_inst;
  ps.resize(n);
  for (int i = 0; i < n; ++i) {
    gpe_status st = check_params(&prms[i]);
    if (st != GPE_OK) return st;
    st = check_knots(ramps[i].n_knots, ramps[i].knot_t, ramps[i].knot_delta, "ramp");
    if (st != GPE_OK) return st;
    if (!std::isfinite(ramps[i].omega)) return fail(GPE_ERR_ARG, "ramp %d: omega must be finite", i);
    if (ramps[i].kind != 0 && ramps[i].kind != GPE_POT_RF_RAMP && ramps[i].kind != GPE_POT_SHELL_RAMP)
      return fail(GPE_ERR_ARG, "ramp %d: kind must be GPE_POT_RF_RAMP (or 0) or GPE_POT_SHELL_RAMP", i);
    gpe_potential pot;
    pot.kind = ramps[i].kind == GPE_POT_SHELL_RAMP ? GPE_POT_SHELL_RAMP : GPE_POT_RF_RAMP;
    pot.n_knots = ramps[i].n_knots;
    pot.field = nullptr;
    pot.omega = ramps[i].omega;
    pot.knot_t = ramps[i].knot_t;
    pot.knot_delta = ramps[i].knot_delta;
    ps[i] = make_params(&pot, &prms[i], t0);
  }
  return GPE_OK;
}

gpe_status gpe_batch_real_time(gpe_batch b, gpe_dtype dtype, void* psi, const void* field, const gpe_ramp* ramps,
                               const gpe_params* prms, double t0, int64_t nsteps, int32_t use_graph, void* work,
                               size_t work_bytes, void* stream, gpe_obs* final_host) {
  if (!b) return fail(GPE_ERR_ARG, "batch is NULL");
  gpe_status st = check_dtype(dtype);
  if (st == GPE_OK) st = check_ptr(psi, "psi");
  if (st == GPE_OK) st = check_ptr(field, "field");
  if (st != GPE_OK) return st;
  if (nsteps < 0 || !std::isfinite(t0)) return fail(GPE_ERR_ARG, "nsteps must be >= 0 and t0 finite");
  std::vector<InstParams> ps;
  st = batch_params(b, ramps, prms, t0, ps);
  if (st != GPE_OK) return st;
  const int integ = prms[0].integrator;
  for (int i = 1; i < b->prob->n_inst; ++i)
    if (prms[i].integrator != integ) return fail(GPE_ERR_ARG, "every instance must use the same integrator");
  st = check_work(work, work_bytes, work_bytes_for(b->prob->total, dtype, rt_work_mode(integ), nsteps, 0));
  if (st != GPE_OK) return st;
  DeviceGuard dg(b->device);
  hipStream_t s = (hipStream_t)stream;
  Ctx c;
  st = make_ctx(b->prob.get(), b->prob->config, s, c);
  if (st != GPE_OK) return st;
  Ordered ord(b->prob.get(), s);
  if (ord.st != GPE_OK) return ord.st;
  st = b->prob->upload(*c.cs, ps, s);
  if (st != GPE_OK) return st;
  bool check = false;
  for (int i = 0; i < b->prob->n_inst; ++i) check = check || !prms[i].skip_stability_check;
  if (check) {
    st = dtype == GPE_C128 ? rt_stability<double>(c, ps.data(), field, psi, integ)
                           : rt_stability<float>(c, ps.data(), field, psi, integ);
    if (st != GPE_OK) return st;
  }
  if (use_graph) {
    st = dtype == GPE_C128 ? batch_rt_graph<double>(c, dtype, psi, field, nsteps, work, integ)
                           : batch_rt_graph<float>(c, dtype, psi, field, nsteps, work, integ);
  } else {
    st = dtype == GPE_C128 ? drive_rt<double>(c, psi, field, nsteps, work, 0, nullptr, integ)
                           : drive_rt<float>(c, psi, field, nsteps, work, 0, nullptr, integ);
  }
  if (st != GPE_OK) return st;
  if (final_host) {
    // observation at the final time t0 + nsteps dt
    st = dtype == GPE_C128 ? drive_observe<double>(c, psi, field, false, nsteps)
                           : drive_observe<float>(c, psi, field, false, nsteps);
    if (st != GPE_OK) return st;
    return read_obs(*b->prob, final_host, s);
  }
  return GPE_OK;
}

gpe_status gpe_batch_fidelity_grad(gpe_batch b, gpe_dtype dtype, const void* psi0, const void* psi_target,
                                   const void* field, const gpe_ramp* ramps, const gpe_params* prms, double t0,
                                   int64_t nsteps, int64_t ckpt_every, int32_t use_graph, void* work,
                                   size_t work_bytes, void* stream, double* loss_host, double* grad_host) {
  if (!b) return fail(GPE_ERR_ARG, "batch is NULL");
  gpe_status st = check_dtype(dtype);
  if (st == GPE_OK) st = check_ptr(psi0, "psi0");
  if (st == GPE_OK) st = check_ptr(psi_target, "psi_target");
  if (st == GPE_OK) st = check_ptr(field, "field");
  if (st != GPE_OK) return st;
  if (!loss_host || !grad_host) return fail(GPE_ERR_ARG, "loss_host and grad_host are required");
  if (nsteps < 1 || ckpt_every < 0 || !std::isfinite(t0)) return fail(GPE_ERR_ARG, "bad nsteps/ckpt_every/t0");
  std::vector<InstParams> ps;
  st = batch_params(b, ramps, prms, t0, ps);
  if (st != GPE_OK) return st;
  for (int i = 0; i < b->prob->n_inst; ++i)
    if (prms[i].integrator != GPE_RK4) return fail(GPE_ERR_ARG, "the fidelity gradient is the adjoint of RK4 only");
  st = check_work(work, work_bytes, work_bytes_for(b->prob->total, dtype, GPE_MODE_ADJ, nsteps, ckpt_every));
  if (st != GPE_OK) return st;
  DeviceGuard dg(b->device);
  hipStream_t s = (hipStream_t)stream;
  Ctx c;
  st = make_ctx(b->prob.get(), b->prob->config, s, c);
  if (st != GPE_OK) return st;
  Ordered ord(b->prob.get(), s);
  if (ord.st != GPE_OK) return ord.st;
  st = b->prob->upload(*c.cs, ps, s);
  if (st != GPE_OK) return st;
  bool check = false;
  for (int i = 0; i < b->prob->n_inst; ++i) check = check || !prms[i].skip_stability_check;
  if (check) {
    st = dtype == GPE_C128 ? rt_stability<double>(c, ps.data(), field, psi0, GPE_RK4, 3.0)
                           : rt_stability<float>(c, ps.data(), field, psi0, GPE_RK4, 3.0);
    if (st != GPE_OK) return st;
  }
  st = dtype == GPE_C128
           ? drive_adjoint<double>(c, psi0, psi_target, field, nsteps, ckpt_every, work, nullptr, use_graph != 0)
           : drive_adjoint<float>(c, psi0, psi_target, field, nsteps, ckpt_every, work, nullptr, use_graph != 0);
  if (st != GPE_OK) return st;
  HIP_TRY(hipStreamSynchronize(s));
  return read_loss_grad(*b->prob, loss_host, grad_host, 0);
}

// ---- launch configuration -------------------------------------------------

int32_t gpe_config_count(void) { return config_count(); }

gpe_status gpe_config_describe(int32_t config, int32_t* block, int32_t* spt, int32_t* xcd, int32_t* rk_scheme,
                               int32_t* nontemporal, int32_t* lds_stage) {
  if (config < 0 || config >= config_count()) return fail(GPE_ERR_ARG, "config %d out of range", config);
  LaunchConfig c = config_get(config);
  if (block) *block = c.block;
  if (spt) *spt = c.spt;
  if (xcd) *xcd = c.xcd;
  if (rk_scheme) *rk_scheme = c.scheme;
  if (nontemporal) *nontemporal = c.nt;
  if (lds_stage) *lds_stage = c.stage;
  return GPE_OK;
}

gpe_status gpe_grid_set_config(gpe_grid g, int32_t config) {
  gpe_status st = check_grid(g);
  if (st != GPE_OK) return st;
  if (config < 0 || config >= config_count()) return fail(GPE_ERR_ARG, "config %d out of range", config);
  g->prob->config = config;
  DeviceGuard dg(g->device);
  return prepare_tables(g->prob.get());
}

gpe_status gpe_grid_get_config(gpe_grid g, int32_t* config) {
  gpe_status st = check_grid(g);
  if (st != GPE_OK) return st;
  if (!config) return fail(GPE_ERR_ARG, "config is NULL");
  *config = g->prob->config;
  return GPE_OK;
}

gpe_status gpe_batch_set_config(gpe_batch b, int32_t config) {
  if (!b) return fail(GPE_ERR_ARG, "batch is NULL");
  if (config < 0 || config >= config_count()) return fail(GPE_ERR_ARG, "config %d out of range", config);
  b->prob->config = config;
  DeviceGuard dg(b->device);
  return prepare_tables(b->prob.get());
}

// Autotuning results, shared by every grid and batch of the process: keyed by
// the element type, the phase, the size class floor(log2 n_active), the class
// floor(log2 mean segment length) (the two properties that decide which
// launch variant streams a layout best) and, for batches, the class
// floor(log2 instance count) (-1 for single grids).
static std::mutex g_tune_mu;
static std::map<std::tuple<int, int, int, int, int>, int> g_tune_cache;

static int log2_class(double v) {
  int b = 0;
  while ((double)(int64_t(1) << (b + 1)) <= v) ++b;
  return b;
}

static std::tuple<int, int, int, int, int> tune_key(const Problem& P, int dtype, int mode, int batch) {
  const double mean_seg = (double)P.total / (double)std::max<int64_t>(1, P.n_segs);
  return std::make_tuple(dtype, mode, log2_class((double)P.total), log2_class(mean_seg),
                         batch ? log2_class((double)P.n_inst) : -1);
}

static gpe_status check_tune_mode(int mode) {
  if (mode != GPE_MODE_RT && mode != GPE_MODE_ITP && mode != GPE_MODE_ITP_REAL)
    return fail(GPE_ERR_ARG, "mode must be GPE_MODE_RT, GPE_MODE_ITP or GPE_MODE_ITP_REAL");
  return GPE_OK;
}

// Time every launch variant on `reps` steps: three interleaved rounds over all
// variants, each variant keeping its fastest round (robust to clock and
// neighbour noise); one untimed step per variant first builds its tables (and
// captures its graph).  `run(ctx, steps)` advances the caller's state.  The
// problem's configuration is set to each variant while it runs (captured
// graphs are keyed by it) and finally to the fastest one.
}  // extern "C"

template <typename Params, typename Run>
static gpe_status tune_variants(Problem* P, hipStream_t s, int reps, Params params, Run run, int* best_out,
                                double* times_ms) {
  const int prev = P->config;
  const int nc = config_count();
  std::vector<double> tmin(nc, 1e300);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(GPE_ERR_DEVICE, "hipEventCreate failed");
  }
  gpe_status st = GPE_OK;
  for (int round = 0; round < 3 && st == GPE_OK; ++round) {
    for (int k = 0; k < nc; ++k) {
      Ctx c;
      P->config = k;
      st = make_ctx(P, k, s, c);
      if (st != GPE_OK) break;
      std::vector<InstParams> ps = params();
      st = P->upload(*c.cs, ps, s);
      if (st != GPE_OK) break;
      st = run(c, 1);
      if (st != GPE_OK) break;
      if (hipEventRecord(e0, s) != hipSuccess) {
        st = fail(GPE_ERR_DEVICE, "hipEventRecord");
        break;
      }
      st = run(c, reps);
      if (st != GPE_OK) break;
      float ms = 0.f;
      if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        st = fail(GPE_ERR_DEVICE, "event timing failed");
        break;
      }
      tmin[k] = std::min(tmin[k], (double)ms / reps);
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != GPE_OK) {
    P->config = prev;
    return st;
  }
  double best = 1e300;
  int bi = prev;
  for (int k = 0; k < nc; ++k) {
    if (times_ms) times_ms[k] = tmin[k];
    if (tmin[k] < best) {
      best = tmin[k];
      bi = k;
    }
  }
  P->config = bi;
  *best_out = bi;
  return GPE_OK;
}

extern "C" {

gpe_status gpe_grid_autotune(gpe_grid g, gpe_dtype dtype, int32_t mode, void* psi, const gpe_potential* pot,
                             const gpe_params* prm, int32_t reps, void* work, size_t work_bytes, void* stream,
                             int32_t* best_config, double* times_ms) {
  gpe_status st = check_grid(g);
  if (st == GPE_OK) st = check_dtype(dtype);
  if (st == GPE_OK) st = check_tune_mode(mode);
  if (st == GPE_OK) st = check_ptr(psi, "psi");
  if (st == GPE_OK) st = check_pot(pot);
  if (st == GPE_OK) st = check_params(prm);
  if (st != GPE_OK) return st;
  if (reps < 1) return fail(GPE_ERR_ARG, "reps must be >= 1");
  const bool itp = mode != GPE_MODE_RT, real = mode == GPE_MODE_ITP_REAL;
  if (itp && prm->integrator != GPE_RK4) return fail(GPE_ERR_ARG, "params.integrator must be 0 for imaginary time");
  st = check_work(work, work_bytes,
                  work_bytes_for(g->lay.n_active, dtype, itp ? mode : rt_work_mode(prm->integrator), reps, 0));
  if (st != GPE_OK) return st;
  // `steps` steps of the tuned phase with the context's launch variant
  auto run = [&](const Ctx& c, int64_t steps) {
    if (itp)
      return dtype == GPE_C128 ? drive_itp<double>(c, psi, pot->field, steps, work, 0, nullptr, real)
                               : drive_itp<float>(c, psi, pot->field, steps, work, 0, nullptr, real);
    return dtype == GPE_C128 ? drive_rt<double>(c, psi, pot->field, steps, work, 0, nullptr, prm->integrator)
                             : drive_rt<float>(c, psi, pot->field, steps, work, 0, nullptr, prm->integrator);
  };
  auto params = [&]() { return std::vector<InstParams>{make_params(pot, prm, 0.0)}; };
  DeviceGuard dg(g->device);
  hipStream_t s = (hipStream_t)stream;
  Ordered ord(g->prob.get(), s);
  if (ord.st != GPE_OK) return ord.st;
  int bi = 0;
  st = tune_variants(g->prob.get(), s, reps, params, run, &bi, times_ms);
  if (st != GPE_OK) return st;
  if (best_config) *best_config = bi;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_cache[tune_key(*g->prob, dtype, mode, 0)] = bi;
  return GPE_OK;
}

gpe_status gpe_grid_apply_tuned(gpe_grid g, gpe_dtype dtype, int32_t mode, int32_t* config) {
  gpe_status st = check_grid(g);
  if (st == GPE_OK) st = check_dtype(dtype);
  if (st == GPE_OK) st = check_tune_mode(mode);
  if (st != GPE_OK) return st;
  if (!config) return fail(GPE_ERR_ARG, "config is NULL");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune_cache.find(tune_key(*g->prob, dtype, mode, 0));
  if (it == g_tune_cache.end()) {
    *config = -1;
    return GPE_OK;
  }
  g->prob->config = it->second;
  *config = it->second;
  DeviceGuard dg(g->device);
  return prepare_tables(g->prob.get());
}

gpe_status gpe_batch_get_config(gpe_batch b, int32_t* config) {
  if (!b || !config) return fail(GPE_ERR_ARG, "batch or config is NULL");
  *config = b->prob->config;
  return GPE_OK;
}

gpe_status gpe_batch_autotune(gpe_batch b, gpe_dtype dtype, void* psi, const void* field, const gpe_ramp* ramps,
                              const gpe_params* prms, int32_t reps, int32_t use_graph, void* work, size_t work_bytes,
                              void* stream, int32_t* best_config, double* times_ms) {
  if (!b) return fail(GPE_ERR_ARG, "batch is NULL");
  gpe_status st = check_dtype(dtype);
  if (st == GPE_OK) st = check_ptr(psi, "psi");
  if (st == GPE_OK) st = check_ptr(field, "field");
  if (st != GPE_OK) return st;
  if (reps < 1) return fail(GPE_ERR_ARG, "reps must be >= 1");
  std::vector<InstParams> ps;
  st = batch_params(b, ramps, prms, 0.0, ps);
  if (st != GPE_OK) return st;
  const int integ = prms[0].integrator;
  for (int i = 1; i < b->prob->n_inst; ++i)
    if (prms[i].integrator != integ) return fail(GPE_ERR_ARG, "every instance must use the same integrator");
  st = check_work(work, work_bytes, work_bytes_for(b->prob->total, dtype, rt_work_mode(integ), reps, 0));
  if (st != GPE_OK) return st;
  auto run = [&](const Ctx& c, int64_t steps) {
    if (use_graph)
      return dtype == GPE_C128 ? batch_rt_graph<double>(c, dtype, psi, field, steps, work, integ)
                               : batch_rt_graph<float>(c, dtype, psi, field, steps, work, integ);
    return dtype == GPE_C128 ? drive_rt<double>(c, psi, field, steps, work, 0, nullptr, integ)
                             : drive_rt<float>(c, psi, field, steps, work, 0, nullptr, integ);
  };
  auto params = [&]() { return ps; };
  DeviceGuard dg(b->device);
  hipStream_t s = (hipStream_t)stream;
  Ordered ord(b->prob.get(), s);
  if (ord.st != GPE_OK) return ord.st;
  int bi = 0;
  st = tune_variants(b->prob.get(), s, reps, params, run, &bi, times_ms);
  if (st != GPE_OK) return st;
  if (best_config) *best_config = bi;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_cache[tune_key(*b->prob, dtype, GPE_MODE_RT, 1)] = bi;
  return GPE_OK;
}

gpe_status gpe_batch_apply_tuned(gpe_batch b, gpe_dtype dtype, int32_t* config) {
  if (!b || !config) return fail(GPE_ERR_ARG, "batch or config is NULL");
  gpe_status st = check_dtype(dtype);
  if (st != GPE_OK) return st;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune_cache.find(tune_key(*b->prob, dtype, GPE_MODE_RT, 1));
  if (it == g_tune_cache.end()) {
    *config = -1;
    return GPE_OK;
  }
  b->prob->config = it->second;
  *config = it->second;
  DeviceGuard dg(b->device);
  return prepare_tables(b->prob.get());
}

gpe_status gpe_autotune_cache_clear(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_cache.clear();
  return GPE_OK;
}

// ---- timing ---------------------------------------------------------------

gpe_status gpe_stream_copy(const void* src, void* dst, size_t bytes, void* stream) {
  gpe_status st = check_ptr(src, "src");
  if (st == GPE_OK) st = check_ptr(dst, "dst");
  if (st != GPE_OK) return st;
  if (bytes % 16 != 0) return fail(GPE_ERR_ARG, "bytes (%zu) is not a multiple of 16", bytes);
  const size_t n16 = bytes / 16;
  if ((n16 + 255) / 256 > (size_t)INT32_MAX) return fail(GPE_ERR_ARG, "copy of %zu bytes is too large", bytes);
  const char* a = (const char*)src;
  char* b = (char*)dst;
  if (a < b + bytes && b < a + bytes) return fail(GPE_ERR_ARG, "src and dst overlap");
  LTRY(run_stream_copy(src, dst, n16, (hipStream_t)stream));
  return GPE_OK;
}

gpe_status gpe_timing_enable(int32_t enable) {
  g_tim.enabled = enable != 0;
  return GPE_OK;
}

gpe_status gpe_timing_reset(void) {
  resolve_pending(0);
  for (int f = 0; f < FAM_COUNT; ++f) {
    g_tim.launches[f] = 0;
    g_tim.ms[f] = 0.0;
  }
  return GPE_OK;
}

int32_t gpe_timing_count(void) { return FAM_COUNT; }

const char* gpe_timing_name(int32_t f) { return family_name(f); }

gpe_status gpe_timing_read(int32_t f, int64_t* launches, double* total_ms) {
  if (f < 0 || f >= FAM_COUNT) return fail(GPE_ERR_ARG, "family out of range");
  resolve_pending(0);
  if (launches) *launches = g_tim.launches[f];
  if (total_ms) *total_ms = g_tim.ms[f];
  return GPE_OK;
}

}  // extern "C"

// The batched entry points of include/lbm.h: many independent lattices advanced by one
// launch per step, with direct launches or captured HIP graphs, and the autotuner that
// picks the schedule.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "handle.h"
#include "kernels.h"
#include "lbm.h"
#include "plan.h"
#include "trace.h"

using namespace lbm;

namespace {

std::string g_batch_create_error;

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

// SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): the generator of the shuffled tile
// orders.
uint64_t splitmix64(uint64_t& s) {
  uint64_t z = (s += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

constexpr int kMaxGraphs = 16;

}  // namespace

struct lbm_batch_t {
  std::vector<lbm_t*> m;
  int32_t max_record = 0;
  int precision = 0;
  int64_t total_tiles = 0, total_box = 0, total_fluid = 0, total_nodes = 0;
  int64_t max_tiles = 0;  // tile-list capacity: the most tiles of the three tile shapes
  std::vector<int32_t> tile_inst, tile_local, box_inst, box_local;
  std::vector<int> nj0;  // box-sweep blocks of each member at create (the lists' sizes)
  std::vector<BatchInst> desc;  // the instance table as last uploaded
  size_t off_desc = 0, off_ti = 0, off_tl = 0, off_bi = 0, off_bl = 0, off_ctl = 0,
         off_ring = 0, off_alt = 0, total = 0;
  // Strip-slot tables of the members that run in the batch in a tile shape other than
  // their own (schedule tile_shape): element offset in the region at off_alt (or -1),
  // tiles along x and y, and the plan generation each was built from.
  std::vector<int64_t> alt_at;
  std::vector<int32_t> alt_ntx, alt_nty, alt_host;
  std::vector<uint64_t> alt_gen;
  char* ws = nullptr;
  hipStream_t stream = nullptr, cap_stream = nullptr;
  bool bound = false;
  int cus = 0;
  int bpar = 0;  // buf[bpar] of every instance-table entry is the member's current state
  lbm_batch_schedule sched{0, 0, 0, 0, LBM_TILE_AUTO};
  // (launches, parity, forces, some body in motion): the last selects the kernel variant
  std::map<std::tuple<int, int, int, int>, hipGraphExec_t> graphs;
  int64_t nrec = 0, steps_done = 0;
  std::vector<uint32_t> rec_scheme;
  std::string err;

  int fail(int code, const std::string& msg) {
    err = msg;
    return code;
  }
  int hip_fail(hipError_t e, const char* what) {
    err = std::string(what) + ": " + hipGetErrorString(e);
    return LBM_EHIP;
  }
  double* ring() const { return reinterpret_cast<double*>(ws + off_ring); }
  int nred() const { return (int(m.size()) + 7) / 8 * 8; }

  void drop_graphs() {
    for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
    graphs.clear();
  }

  // Tile and box-sweep lists: instance-major, the tile list optionally shuffled.
  // A member's box sweep may not change size after create (lbm_set_mask with a resized
  // box): the lists and their workspace are sized for the sizes at create.
  bool sizes_kept() const {
    for (size_t i = 0; i < m.size(); ++i)
      if (m[i]->njblocks != nj0[i]) return false;
    return true;
  }

  // Tile rows of member i in the batch, and its tile count in tiles of `rows` rows.
  int rows_of(size_t i) const {
    if (sched.tile_shape == LBM_TILE_AUTO) return m[i]->plan.tile_rows;
    return sched.tile_shape == LBM_TILE_NARROW ? 4 : 1;
  }
  static int64_t tiles_in(const Plan& p, int rows) {
    const int tile_w = kTileW / rows;
    return int64_t((p.nx + tile_w - 1) / tile_w) * ((p.ny + rows - 1) / rows);
  }

  // The strip-slot tables of the members whose batch tile shape differs from their own
  // (each member's own table serves the others), from the members' present plans.
  void build_alt() {
    alt_at.assign(m.size(), -1);
    alt_ntx.assign(m.size(), 0);
    alt_nty.assign(m.size(), 0);
    alt_gen.assign(m.size(), 0);
    alt_host.clear();
    std::vector<int32_t> tab;
    for (size_t i = 0; i < m.size(); ++i) {
      alt_gen[i] = m[i]->plan_gen;
      const int rows = rows_of(i);
      if (rows == m[i]->plan.tile_rows) continue;
      tile_slots(m[i]->plan, rows, alt_ntx[i], alt_nty[i], tab);
      alt_at[i] = int64_t(alt_host.size());
      alt_host.insert(alt_host.end(), tab.begin(), tab.end());
    }
  }
  bool alt_current() const {
    if (alt_gen.size() != m.size()) return false;
    for (size_t i = 0; i < m.size(); ++i)
      if (alt_gen[i] != m[i]->plan_gen) return false;
    return true;
  }

  void build_lists() {
    tile_inst.clear();
    tile_local.clear();
    box_inst.clear();
    box_local.clear();
    // Instance order of the tile list: as given, or largest first for the tile queue
    // (the longest instances start first; ties keep the given order).
    std::vector<size_t> order(m.size());
    for (size_t i = 0; i < m.size(); ++i) order[i] = i;
    if (sched.tile_queue)
      std::stable_sort(order.begin(), order.end(), [&](size_t p, size_t q) {
        return int64_t(m[p]->g.nx) * m[p]->g.ny > int64_t(m[q]->g.nx) * m[q]->g.ny;
      });
    for (size_t i : order) {
      const int64_t nt = tiles_in(m[i]->plan, rows_of(i));
      for (int64_t t = 0; t < nt; ++t) {
        tile_inst.push_back(int32_t(i));
        tile_local.push_back(int32_t(t));
      }
    }
    total_tiles = int64_t(tile_inst.size());
    for (size_t i = 0; i < m.size(); ++i)
      for (int t = 0; t < m[i]->njblocks; ++t) {
        box_inst.push_back(int32_t(i));
        box_local.push_back(t);
      }
    if (sched.tile_order != 0) {
      uint64_t s = sched.tile_order;
      for (size_t k = tile_inst.size(); k > 1; --k) {
        const size_t j = size_t(splitmix64(s) % k);
        std::swap(tile_inst[k - 1], tile_inst[j]);
        std::swap(tile_local[k - 1], tile_local[j]);
      }
    }
  }

  // Instance table for the members' present state, with buf[bpar] the current buffer.
  std::vector<BatchInst> make_desc() const {
    std::vector<BatchInst> d(m.size());
    for (size_t i = 0; i < m.size(); ++i) {
      const lbm_t* h = m[i];
      BatchInst& e = d[i];
      std::memset(static_cast<void*>(&e), 0, sizeof(BatchInst));
      e.a = step_args(h);
      if (i < alt_at.size() && alt_at[i] >= 0) {
        // This member runs in the batch's tile shape, with its slots in that tile order.
        e.a.tile_rows = rows_of(i);
        e.a.ntx = alt_ntx[i];
        e.a.nty = alt_nty[i];
        e.a.ntiles = alt_ntx[i] * alt_nty[i];
        e.a.strip_slot = reinterpret_cast<const int32_t*>(ws + off_alt) + alt_at[i];
      }
      for (int j = 0; j < 2; ++j) e.buf[j] = h->buf(h->cur ^ j ^ bpar);
      e.part[0] = h->part(0);
      e.part[1] = h->part(1);
      e.ring = ring() + int64_t(i) * kRingRow;
      e.step_off = h->steps_done - steps_done;
      if (h->plan.has_box) {
        e.box = box_args(h, nullptr);
        e.njblocks = h->njblocks;
      }
      // The batch reads each motion from its own table, which it uploads in order on
      // its stream, not from the member's copy (written on the member's stream).
      const BodyMotion* mot = nullptr;
      if (h->motion.moving) {
        e.mot.ux = h->motion.ux;
        e.mot.uy = h->motion.uy;
        e.mot.omega = h->motion.omega;
        e.mot.xc = h->motion.xc;
        e.mot.yc = h->motion.yc;
        e.mot.moving = 1;
        mot = reinterpret_cast<const BodyMotion*>(ws + off_desc + i * sizeof(BatchInst) +
                                                  offsetof(BatchInst, mot));
      }
      e.a.motion = mot;
      e.box.motion = h->plan.has_box ? mot : nullptr;
    }
    return d;
  }

  BatchLaunch launch() const {
    BatchLaunch L{};
    L.inst = reinterpret_cast<const BatchInst*>(ws + off_desc);
    L.tile_inst = reinterpret_cast<const int32_t*>(ws + off_ti);
    L.tile_local = reinterpret_cast<const int32_t*>(ws + off_tl);
    L.box_inst = reinterpret_cast<const int32_t*>(ws + off_bi);
    L.box_local = reinterpret_cast<const int32_t*>(ws + off_bl);
    L.ctl = reinterpret_cast<const int32_t*>(ws + off_ctl);
    // The tile counters sit in the control word's block, after its four words.
    L.queue = sched.tile_queue && sched.grid_blocks > 0
                  ? reinterpret_cast<int32_t*>(ws + off_ctl) + 4 : nullptr;
    L.n_inst = int32_t(m.size());
    L.nred = nred();
    L.total_tiles = int32_t(total_tiles);
    L.total_box_blocks = int32_t(total_box);
    L.grid_blocks = sched.grid_blocks > 0 ? (sched.grid_blocks + 7) / 8 * 8 : 0;
    L.collision = m[0]->g.collision;
    L.moving = 0;
    for (const lbm_t* h : m) L.moving |= h->motion.moving;
    return L;
  }

  int upload(const void* host, size_t off, size_t bytes, const char* what) {
    if (bytes == 0) return LBM_OK;
    const hipError_t e = hipMemcpyAsync(ws + off, host, bytes, hipMemcpyHostToDevice, stream);
    return e == hipSuccess ? LBM_OK : hip_fail(e, what);
  }

  int upload_lists() {
    int rc = upload(tile_inst.data(), off_ti, tile_inst.size() * 4, "upload tile list");
    if (rc == LBM_OK)
      rc = upload(alt_host.data(), off_alt, alt_host.size() * 4, "upload strip slots");
    if (rc == LBM_OK) rc = upload(tile_local.data(), off_tl, tile_local.size() * 4, "upload tile list");
    if (rc == LBM_OK) rc = upload(box_inst.data(), off_bi, box_inst.size() * 4, "upload box list");
    if (rc == LBM_OK) rc = upload(box_local.data(), off_bl, box_local.size() * 4, "upload box list");
    if (rc != LBM_OK) return rc;
    const hipError_t e = hipStreamSynchronize(stream);
    return e == hipSuccess ? LBM_OK : hip_fail(e, "upload synchronize");
  }

  // Take schedule s; the tile list (and the strip-slot tables of a tile shape) are
  // rebuilt and uploaded when the order or the shape changes.
  int use_schedule(const lbm_batch_schedule& s) {
    const bool reorder = s.tile_order != sched.tile_order || s.tile_queue != sched.tile_queue ||
                         s.tile_shape != sched.tile_shape;
    sched = s;
    if (!reorder) return LBM_OK;
    build_alt();
    build_lists();
    return bound ? upload_lists() : LBM_OK;
  }

  // Bring the device instance table up to date with the members (a member stepped,
  // re-bound or given a new tau since the last call).
  int refresh() {
    for (const lbm_t* h : m)
      if (!h->bound) return fail(LBM_ESTATE, "a member is no longer bound");
    if (!sizes_kept())
      return fail(LBM_ESTATE, "a member's control volume changed size; create a new batch");
    if (!alt_current()) {
      // A member's plan changed (a mask change): its slots in the batch's tile order too.
      build_alt();
      const int rc = upload(alt_host.data(), off_alt, alt_host.size() * 4, "upload strip slots");
      if (rc != LBM_OK) return rc;
    }
    std::vector<BatchInst> d = make_desc();
    if (d.size() == desc.size() &&
        std::memcmp(d.data(), desc.data(), d.size() * sizeof(BatchInst)) == 0)
      return LBM_OK;
    // The previous upload may still be read by queued kernels; the copy is ordered
    // after them, and the host copy is kept until the stream has consumed it.
    desc.swap(d);
    int rc = upload(desc.data(), off_desc, desc.size() * sizeof(BatchInst), "upload instances");
    if (rc != LBM_OK) return rc;
    const hipError_t e = hipStreamSynchronize(stream);
    return e == hipSuccess ? LBM_OK : hip_fail(e, "upload synchronize");
  }

  // Graph of `len` consecutive step launches starting at buffer parity `parity`.
  int graph(int len, int parity, bool forces, hipGraphExec_t* out) {
    const BatchLaunch L = launch();
    const auto key = std::make_tuple(len, parity, forces ? 1 : 0, int(L.moving));
    auto it = graphs.find(key);
    if (it != graphs.end()) {
      *out = it->second;
      return LBM_OK;
    }
    if (int(graphs.size()) >= kMaxGraphs) drop_graphs();
    hipError_t e = hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "begin graph capture");
    hipError_t le = hipSuccess;
    for (int k = 0; k < len && le == hipSuccess; ++k)
      le = launch_batch_step(precision, forces, L, (parity + k) & 1, k, cap_stream);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cap_stream, &g);
    if (le != hipSuccess || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return hip_fail(le != hipSuccess ? le : e, "capture batch steps");
    }
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "instantiate batch graph");
    graphs[key] = x;
    *out = x;
    return LBM_OK;
  }

  // Enqueue n >= 1 steps of every instance; with forces, step k's row goes to ring row
  // row0 + k of every instance.
  int enqueue(int32_t n, bool forces, int64_t row0) {
    int rc = refresh();
    if (rc != LBM_OK) return rc;
    const BatchLaunch L = launch();
    const int G = sched.graph_steps;
    if (L.queue) {
      const hipError_t e = launch_batch_queue_reset(L.queue, stream);
      if (e != hipSuccess) return hip_fail(e, "reset tile queue");
    }
    int32_t done = 0;
    while (done < n) {
      const int len = G > 0 ? std::min<int32_t>(G, n - done) : n - done;
      hipError_t e;
      if (forces || precision == LBM_FP32SR) {
        e = launch_batch_ctl(reinterpret_cast<int32_t*>(ws + off_ctl), int32_t(row0 + done), done,
                             steps_done, stream);
        if (e != hipSuccess) return hip_fail(e, "launch batch control");
      }
      if (G > 0) {
        hipGraphExec_t x = nullptr;
        rc = graph(len, bpar, forces, &x);
        if (rc != LBM_OK) return rc;
        e = hipGraphLaunch(x, stream);
        if (e != hipSuccess) return hip_fail(e, "launch batch graph");
      } else {
        for (int k = 0; k < len; ++k) {
          e = launch_batch_step(precision, forces, L, (bpar + k) & 1, k, stream);
          if (e != hipSuccess) return hip_fail(e, "launch batch step");
        }
      }
      bpar = (bpar + len) & 1;
      done += len;
    }
    if (forces) {
      const hipError_t e = launch_batch_tail(precision, L, bpar, int32_t(row0 + n - 1),
                                             (n - 1) & 1, n >= 2, stream);
      if (e != hipSuccess) return hip_fail(e, "launch batch tail");
    }
    for (lbm_t* h : m) {
      h->cur = (h->cur + n) & 1;
      h->steps_done += n;
      h->adj_valid = false;
    }
    steps_done += n;
    // The table is unchanged: buf[bpar] is again every member's current buffer.
    return LBM_OK;
  }
};

extern "C" {

int lbm_batch_create(lbm_t* const* members, int32_t n, int32_t max_record, lbm_batch_t** out) {
  g_batch_create_error.clear();
  if (!out || !members || n < 1 || max_record < 1) {
    g_batch_create_error = "need members, n >= 1, max_record >= 1 and an output pointer";
    return LBM_EINVAL;
  }
  *out = nullptr;
  std::vector<lbm_t*> m(members, members + n);
  for (int i = 0; i < n; ++i) {
    if (!m[i] || !m[i]->bound) {
      g_batch_create_error = "member " + std::to_string(i) + " is null or unbound";
      return LBM_EINVAL;
    }
    if (m[i]->g.precision != m[0]->g.precision) {
      g_batch_create_error = "members differ in precision";
      return LBM_EINVAL;
    }
    if (m[i]->g.collision != m[0]->g.collision) {
      g_batch_create_error = "members differ in collision operator";
      return LBM_EINVAL;
    }
    if (m[i]->buf_bytes32() == 0) {
      g_batch_create_error = "member " + std::to_string(i) + " has a state buffer of 4 GiB or more";
      return LBM_EINVAL;
    }
  }
  {
    std::vector<lbm_t*> s = m;
    std::sort(s.begin(), s.end());
    if (std::adjacent_find(s.begin(), s.end()) != s.end()) {
      g_batch_create_error = "a member appears twice";
      return LBM_EINVAL;
    }
  }
  lbm_batch_t* b = new (std::nothrow) lbm_batch_t();
  if (!b) return LBM_ENOMEM;
  b->m = m;
  b->max_record = max_record;
  b->precision = m[0]->g.precision;
  int64_t alt_cap = 0;
  for (const lbm_t* h : m) {
    const int64_t wide = lbm_batch_t::tiles_in(h->plan, 1), narrow = lbm_batch_t::tiles_in(h->plan, 4);
    b->total_tiles += h->plan.ntiles;
    b->max_tiles += std::max(wide, narrow);
    alt_cap += std::max(wide, narrow) * kStrips;
    b->total_box += h->njblocks;
    b->nj0.push_back(h->njblocks);
    b->total_fluid += h->plan.n_fluid;
    b->total_nodes += int64_t(h->plan.nx) * h->plan.ny;
  }
  if (b->max_tiles >= (int64_t(1) << 31) || b->total_box >= (int64_t(1) << 31) ||
      alt_cap >= (int64_t(1) << 31)) {
    delete b;
    g_batch_create_error = "too many tiles";
    return LBM_ENOMEM;
  }
  b->build_alt();
  b->build_lists();
  size_t off = 0;
  b->off_desc = off;
  off = align256(off + size_t(n) * sizeof(BatchInst));
  b->off_ti = off;
  off = align256(off + size_t(b->max_tiles) * 4);
  b->off_tl = off;
  off = align256(off + size_t(b->max_tiles) * 4);
  b->off_alt = off;
  off = align256(off + size_t(alt_cap) * 4);
  b->off_bi = off;
  off = align256(off + size_t(b->total_box) * 4);
  b->off_bl = off;
  off = align256(off + size_t(b->total_box) * 4);
  b->off_ctl = off;
  off = align256(off + 8 * sizeof(int32_t));  // control words, then the two tile counters
  b->off_ring = off;
  off = align256(off + size_t(n) * size_t(max_record) * kRingRow * sizeof(double));
  b->total = off;
  *out = b;
  return LBM_OK;
}

int lbm_batch_workspace_bytes(const lbm_batch_t* b, size_t* bytes) {
  if (!b || !bytes) return LBM_EINVAL;
  *bytes = b->total;
  return LBM_OK;
}

int lbm_batch_bind(lbm_batch_t* b, void* device_workspace, size_t bytes, void* hip_stream) {
  if (!b) return LBM_EINVAL;
  if (!device_workspace) return b->fail(LBM_EINVAL, "null workspace");
  if (reinterpret_cast<uintptr_t>(device_workspace) % 256)
    return b->fail(LBM_EINVAL, "workspace must be 256-byte aligned");
  if (bytes < b->total) return b->fail(LBM_ENOMEM, "workspace smaller than lbm_batch_workspace_bytes");
  b->drop_graphs();
  b->ws = static_cast<char*>(device_workspace);
  b->stream = static_cast<hipStream_t>(hip_stream);
  if (!b->cap_stream) {
    const hipError_t e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return b->hip_fail(e, "create capture stream");
  }
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return b->hip_fail(e, "query compute units");
  b->bpar = 0;
  b->desc.clear();
  b->nrec = 0;
  b->rec_scheme.clear();
  int rc = b->upload_lists();
  if (rc == LBM_OK) rc = b->refresh();
  if (rc != LBM_OK) return rc;
  b->bound = true;
  return LBM_OK;
}

int lbm_batch_set_schedule(lbm_batch_t* b, const lbm_batch_schedule* s) {
  if (!b || !s) return LBM_EINVAL;
  if (s->grid_blocks < 0 || s->graph_steps < 0 || (s->graph_steps & 1))
    return b->fail(LBM_EINVAL, "grid_blocks and graph_steps must be >= 0, graph_steps even");
  if (s->tile_queue != 0 && s->tile_queue != 1)
    return b->fail(LBM_EINVAL, "tile_queue must be 0 or 1");
  if (s->tile_queue && s->grid_blocks == 0)
    return b->fail(LBM_EINVAL, "the tile queue needs a persistent grid (grid_blocks > 0)");
  if (s->tile_shape != LBM_TILE_AUTO && s->tile_shape != LBM_TILE_WIDE &&
      s->tile_shape != LBM_TILE_NARROW)
    return b->fail(LBM_EINVAL, "unknown tile shape");
  const bool reorder = s->tile_order != b->sched.tile_order ||
                       s->tile_queue != b->sched.tile_queue || s->tile_shape != b->sched.tile_shape;
  if (reorder && !b->sizes_kept())
    return b->fail(LBM_ESTATE, "a member's control volume changed size; create a new batch");
  b->drop_graphs();
  return b->use_schedule(*s);
}

int lbm_batch_step(lbm_batch_t* b, int32_t n, uint32_t force_scheme) {
  lbm::TraceRange range("lbm_batch_step");
  if (!b) return LBM_EINVAL;
  if (!b->bound) return b->fail(LBM_ESTATE, "batch is not bound to a workspace");
  if (n < 0) return b->fail(LBM_EINVAL, "n must be >= 0");
  if (force_scheme & ~LBM_FORCE_ALL) return b->fail(LBM_EINVAL, "unknown force scheme bits");
  const bool forces = force_scheme != 0;
  if (forces && b->nrec + n > b->max_record)
    return b->fail(LBM_EOVERFLOW, "force ring would overflow; read lbm_batch_forces first");
  if (n == 0) return LBM_OK;
  const int rc = b->enqueue(n, forces, b->nrec);
  if (rc != LBM_OK) return rc;
  if (forces) {
    b->nrec += n;
    b->rec_scheme.insert(b->rec_scheme.end(), size_t(n), force_scheme);
  }
  return LBM_OK;
}

int lbm_batch_autotune(lbm_batch_t* b, int32_t steps, uint32_t force_scheme,
                       lbm_batch_schedule* best, double* ms_per_step) {
  lbm::TraceRange range("lbm_batch_autotune");
  if (!b) return LBM_EINVAL;
  if (!b->bound) return b->fail(LBM_ESTATE, "batch is not bound to a workspace");
  if (steps < 1) return b->fail(LBM_EINVAL, "steps must be >= 1");
  if (force_scheme & ~LBM_FORCE_ALL) return b->fail(LBM_EINVAL, "unknown force scheme bits");
  const bool forces = force_scheme != 0;
  if (forces && b->nrec + steps > b->max_record)
    return b->fail(LBM_EOVERFLOW, "force ring cannot hold the timed steps");
  // Candidates reorder the tile list, which is sized for the members at create.
  if (!b->sizes_kept())
    return b->fail(LBM_ESTATE, "a member's control volume changed size; create a new batch");
  const int gsteps = std::max(2, std::min(64, steps / 2 * 2));
  const int per_cu[] = {0, 1, 2, 4, 8};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return b->hip_fail(e, "create events");
  }
  const lbm_batch_schedule keep = b->sched;
  lbm_batch_schedule win = keep;
  double win_ms = INFINITY;
  // Warm-up of the same length (captures the graphs), then the timed run.
  auto time_candidate = [&](const lbm_batch_schedule& s) -> int {
    b->drop_graphs();
    int r = b->use_schedule(s);
    if (r == LBM_OK) r = b->enqueue(steps, forces, b->nrec);
    if (r != LBM_OK) return r;
    e = hipEventRecord(e0, b->stream);
    if (e == hipSuccess) r = b->enqueue(steps, forces, b->nrec);
    if (r != LBM_OK) return r;
    if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) return b->hip_fail(e, "time candidate");
    const double per = double(ms) / steps;
    if (per < win_ms) {
      win_ms = per;
      win = s;
    }
    return LBM_OK;
  };
  int rc = LBM_OK;
  for (int pc : per_cu) {
    // One workgroup per tile: direct launches or graphs; persistent grids: the same
    // with the static stride and with the tile queue.
    for (int cand = 0; cand < (pc > 0 ? 4 : 2) && rc == LBM_OK; ++cand) {
      lbm_batch_schedule s = keep;
      s.grid_blocks = pc * b->cus;
      s.graph_steps = (cand & 1) ? gsteps : 0;
      s.tile_queue = cand >> 1;
      rc = time_candidate(s);
    }
    if (rc != LBM_OK) break;
  }
  // The fastest schedule with each of the other tile shapes.
  if (rc == LBM_OK) {
    const lbm_batch_schedule base = win;
    for (int shape : {LBM_TILE_AUTO, LBM_TILE_WIDE, LBM_TILE_NARROW}) {
      if (shape == base.tile_shape || rc != LBM_OK) continue;
      lbm_batch_schedule s = base;
      s.tile_shape = shape;
      rc = time_candidate(s);
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->drop_graphs();
  const int rc2 = b->use_schedule(rc == LBM_OK ? win : keep);
  if (rc != LBM_OK) return rc;
  if (rc2 != LBM_OK) return rc2;
  if (best) *best = win;
  if (ms_per_step) *ms_per_step = win_ms;
  return LBM_OK;
}

int lbm_batch_forces(lbm_batch_t* b, double* out, int64_t cap, int64_t* k_out,
                     uint8_t* nonfinite) {
  lbm::TraceRange range("lbm_batch_forces");
  if (!b) return LBM_EINVAL;
  if (!b->bound) return b->fail(LBM_ESTATE, "batch is not bound to a workspace");
  const int64_t k = b->nrec;
  const size_t n = b->m.size();
  if (k_out) *k_out = k;
  if (nonfinite) std::memset(nonfinite, 0, n);
  if (k == 0) return LBM_OK;
  if (!out || cap < k) return b->fail(LBM_EINVAL, "output holds fewer rows than recorded");
  // Rows are step-major ([step][instance][kRingRow]): the k recorded steps are one
  // contiguous block.
  std::vector<double> rows(n * size_t(k) * kRingRow);
  hipError_t e = hipMemcpyAsync(rows.data(), b->ring(), rows.size() * sizeof(double),
                                hipMemcpyDeviceToHost, b->stream);
  if (e != hipSuccess) return b->hip_fail(e, "download force ring");
  e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return b->hip_fail(e, "forces synchronize");
  bool all_finite = true;
  for (size_t i = 0; i < n; ++i) {
    const bool has_box = b->m[i]->plan.has_box;
    bool finite = true;
    for (int64_t t = 0; t < k; ++t)
      finite = row_forces(&rows[(size_t(t) * n + i) * kRingRow], b->rec_scheme[size_t(t)],
                          has_box, out + (int64_t(i) * cap + t) * 2 * kSchemes) && finite;
    if (!finite) {
      all_finite = false;
      if (nonfinite) nonfinite[i] = 1;
    }
  }
  b->nrec = 0;
  b->rec_scheme.clear();
  if (!all_finite) return b->fail(LBM_ENONFINITE, "an instance has a non-finite force");
  return LBM_OK;
}

int lbm_batch_get_info(const lbm_batch_t* b, lbm_batch_info* info) {
  if (!b || !info) return LBM_EINVAL;
  info->n_inst = int32_t(b->m.size());
  info->n_recorded = int32_t(b->nrec);
  info->total_tiles = b->total_tiles;
  info->total_fluid = b->total_fluid;
  info->total_nodes = b->total_nodes;
  info->steps_done = b->steps_done;
  info->n_graphs = int32_t(b->graphs.size());
  info->compute_units = b->cus;
  info->schedule = b->sched;
  return LBM_OK;
}

int lbm_batch_destroy(lbm_batch_t* b) {
  if (!b) return LBM_OK;
  b->drop_graphs();
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  delete b;
  return LBM_OK;
}

const char* lbm_batch_last_error(const lbm_batch_t* b) {
  return b ? b->err.c_str() : g_batch_create_error.c_str();
}

}  // extern "C"

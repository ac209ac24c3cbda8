// C ABI of libccut.so (declarations and contracts in include/ccut.h).
//
// A call runs the hot path of Clifford-based circuit cutting on one GPU:
// per fragment, every variant is evaluated (Clifford: tableau pass to an
// affine sample model, then exact tables or Philox shots; non-Clifford:
// LDS state vector), rewritten in the Pauli basis of each cut axis, and
// the fragment tensors are contracted over the 4^k cut terms.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/ccut.h"
#include "common.hpp"
#include "plan.hpp"

using namespace ccut;

namespace {

// Grow-only pool of device chunks, reset per call: after the first calls of
// a given shape no allocation happens on the hot path.
struct Arena {
  struct Chunk {
    char *p;
    size_t cap, used;
  };
  std::vector<Chunk> chunks;
  ccut_alloc_fn alloc = nullptr;
  ccut_free_fn free_fn = nullptr;
  void *user = nullptr;

  void reset() {
    for (auto &c : chunks) c.used = 0;
    n_uploads = 0;
  }
  bool frozen = false;  // set while a stream capture is open: no allocation then
  // a hash of each upload's bytes in allocation order since the last reset:
  // a re-enqueue that reuses earlier uploads in place checks that its bytes
  // are the same ones (the sequence must repeat exactly)
  std::vector<uint64_t> upload_hash;
  size_t n_uploads = 0;
  void *get(size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    if (bytes == 0) bytes = 256;
    for (auto &c : chunks)
      if (c.cap - c.used >= bytes) {
        void *r = c.p + c.used;
        c.used += bytes;
        return r;
      }
    if (frozen) return nullptr;
    size_t cap = std::max(bytes, size_t(64) << 20);
    void *p = nullptr;
    if (alloc) {
      p = alloc(cap, user);
    } else if (hipMalloc(&p, cap) != hipSuccess) {
      p = nullptr;
    }
    if (!p) return nullptr;
    chunks.push_back({(char *)p, cap, bytes});
    return p;
  }
  void release() {
    for (auto &c : chunks) {
      if (free_fn)
        free_fn(c.p, user);
      else
        (void)hipFree(c.p);
    }
    chunks.clear();
  }
};

struct PendingTiming {
  uint32_t kid;
  hipEvent_t a, b;
};

}  // namespace

struct ccut_ctx {
  int device = -1;
  hipStream_t stream = nullptr;   // the caller's stream: results are ordered on it
  hipStream_t aux = nullptr;      // library stream for non-Clifford fragments (default priority)
  hipStream_t cur = nullptr;      // stream the next launch goes to
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  uint32_t max_nc = 12, max_cuts = 12;
  std::string err;
  std::atomic<int> cancel{0};
  int children = 0;     // plans, batches, term models and networks created from this context
  bool closed = false;  // ccut_ctx_destroy was called while children were alive
  Arena arena;
  bool timing = false;
  std::vector<PendingTiming> pending;
  std::vector<hipEvent_t> event_pool;
  uint64_t launches[CCUT_K_COUNT] = {};
  double total_ms[CCUT_K_COUNT] = {};
  std::vector<std::vector<char>> staged;  // host copies kept alive until the call's final sync
  bool use_aux = true;       // route non-Clifford fragments to the auxiliary stream
  bool replay_uploads = false;  // re-enqueue of an identical sequence: reuse earlier uploads, copy nothing
  // Pinned staging of host-to-device uploads: a ring of slots, one per call;
  // a slot is reused only after the events recorded behind its call's work
  // (on both streams) have completed, so calls with device outputs need not
  // synchronize.
  struct PinSlot {
    std::vector<std::pair<char *, size_t>> chunks;
    size_t chunk = 0, used = 0;
    hipEvent_t ev_s = nullptr, ev_a = nullptr;
    bool pending = false;
  };
  static constexpr int kPinSlots = 4;
  PinSlot pin[kPinSlots];
  int pin_cur = -1;
  // Call graphs: a device-output call repeated with identical arguments is
  // captured once and then replayed.  While a capture is open, uploads go to
  // the captured call's own device block, filled once from its pinned block
  // before the first launch; the graph itself holds kernels only.
  bool call_graphs = true;
  hipStream_t cap_stream = nullptr;  // capture stream of call graphs
  struct CallGraph *capturing = nullptr;
  size_t call_upload_bytes = 0;  // staged bytes of the current call
};

// One captured call: its argument key, the executable graph, and the
// device block holding the call's uploads (with the pinned block they are
// copied from once).
struct CallGraph {
  std::vector<uint8_t> key;
  hipGraphExec_t exec = nullptr;
  char *pin = nullptr;
  char *dev = nullptr;
  size_t pin_cap = 0, pin_used = 0, upload_bytes = 0;
  bool no_graph = false;  // capture failed once: stay eager
  uint64_t last_use = 0;
  void release() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (pin) (void)hipHostFree(pin);
    if (dev) (void)hipFree(dev);
    exec = nullptr;
    pin = nullptr;
    dev = nullptr;
  }
};

struct ccut_plan {
  ccut_ctx *ctx = nullptr;
  PlanData pd;
  std::vector<uint32_t *> d_ops;   // per fragment, uploaded on first evaluation
  std::vector<double *> d_mats;
  std::vector<uint32_t *> d_back;  // Clifford fragments: the carry-back stream
  std::vector<uint32_t> n_back;
  std::vector<uint32_t *> d_layers, d_back_layers;  // layer offsets of both streams
  std::vector<uint32_t> n_layers, n_back_layers;
  std::vector<CallGraph> graphs;  // least recently used first out, at most kMaxCallGraphs
  uint64_t graph_tick = 0;
  static constexpr size_t kMaxCallGraphs = 8;
  ~ccut_plan() {
    // a replay may still be reading the graphs' upload blocks
    if (!graphs.empty() && ctx && ctx->device >= 0) (void)hipStreamSynchronize(ctx->stream);
    for (auto &g : graphs) g.release();
    for (auto p : d_ops)
      if (p) (void)hipFree(p);
    for (auto p : d_mats)
      if (p) (void)hipFree(p);
    for (auto p : d_back)
      if (p) (void)hipFree(p);
    for (auto p : d_layers)
      if (p) (void)hipFree(p);
    for (auto p : d_back_layers)
      if (p) (void)hipFree(p);
  }
};

static thread_local std::string g_create_err;

namespace ccut {
void set_call_error(const char *msg) { g_create_err = msg; }
}  // namespace ccut

namespace {

ccut_status fail(ccut_ctx *ctx, ccut_status st, const std::string &msg) {
  if (ctx) ctx->err = msg;
  return st;
}

#define HIP_TRY(ctx, expr)                                                                      \
  do {                                                                                          \
    hipError_t _e = (expr);                                                                     \
    if (_e != hipSuccess)                                                                       \
      return fail((ctx), CCUT_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(_e));     \
  } while (0)

hipEvent_t take_event(ccut_ctx *c) {
  if (!c->event_pool.empty()) {
    hipEvent_t e = c->event_pool.back();
    c->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets one kernel launch with events on the context stream when timing is on.
struct KTimer {
  ccut_ctx *c;
  uint32_t kid;
  hipEvent_t a = nullptr, b = nullptr;
  KTimer(ccut_ctx *ctx, uint32_t k) : c(ctx), kid(k) {
    if (c->timing) {
      a = take_event(c);
      b = take_event(c);
      if (a) (void)hipEventRecord(a, c->cur);
    }
  }
  ~KTimer() {
    if (c->timing && a && b) {
      (void)hipEventRecord(b, c->cur);
      c->pending.push_back({kid, a, b});
    }
  }
};

template <class T>
T *aget(ccut_ctx *c, size_t count) {
  return (T *)c->arena.get(count * sizeof(T));
}

// Upload each fragment's op streams once per plan: for Clifford fragments
// the fused forward stream and the carry-back stream, for non-Clifford ones
// the state-vector program with its matrices; padded with no-ops
// (identities) to a multiple of 16 words so kernels can fetch ops sixteen at
// a time.
ccut_status ensure_ops(ccut_plan *p) {
  ccut_ctx *c = p->ctx;
  if (!p->d_ops.empty()) return CCUT_OK;
  for (const Fragment &f : p->pd.frags) {
    uint32_t *bk = nullptr;
    std::vector<uint32_t> back = f.cl_back;
    while (back.size() % 16 || back.empty()) back.push_back(pack_op(G_NOP, 0, 0));
    if (f.clifford) {
      HIP_TRY(c, hipMalloc(&bk, back.size() * sizeof(uint32_t)));
      HIP_TRY(c, hipMemcpy(bk, back.data(), back.size() * 4, hipMemcpyHostToDevice));
    }
    p->d_back.push_back(bk);
    p->n_back.push_back((uint32_t)f.cl_back.size());
    uint32_t *dl = nullptr, *dbl = nullptr;
    if (f.clifford) {
      HIP_TRY(c, hipMalloc(&dl, std::max<size_t>(f.cl_layers.size(), 1) * 4));
      HIP_TRY(c, hipMalloc(&dbl, std::max<size_t>(f.cl_back_layers.size(), 1) * 4));
      if (!f.cl_layers.empty())
        HIP_TRY(c, hipMemcpy(dl, f.cl_layers.data(), f.cl_layers.size() * 4, hipMemcpyHostToDevice));
      if (!f.cl_back_layers.empty())
        HIP_TRY(c, hipMemcpy(dbl, f.cl_back_layers.data(), f.cl_back_layers.size() * 4, hipMemcpyHostToDevice));
    }
    p->d_layers.push_back(dl);
    p->d_back_layers.push_back(dbl);
    p->n_layers.push_back(f.cl_layers.empty() ? 0u : (uint32_t)f.cl_layers.size() - 1);
    p->n_back_layers.push_back(f.cl_back_layers.empty() ? 0u : (uint32_t)f.cl_back_layers.size() - 1);
    std::vector<uint32_t> words = f.clifford ? f.cl_words : f.sv_prog;
    std::vector<double> mats = f.clifford ? std::vector<double>() : f.sv_prog_mats;
    while (words.size() % 16 || words.empty()) {
      words.push_back(pack_op(G_NOP, 0, 0));
      if (!f.clifford) mats.insert(mats.end(), 8, 0.0);
    }
    if (mats.empty()) mats.assign(8, 0.0);
    uint32_t *o = nullptr;
    double *t = nullptr;
    HIP_TRY(c, hipMalloc(&o, words.size() * sizeof(uint32_t)));
    HIP_TRY(c, hipMalloc(&t, mats.size() * sizeof(double)));
    HIP_TRY(c, hipMemcpy(o, words.data(), words.size() * 4, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(t, mats.data(), mats.size() * 8, hipMemcpyHostToDevice));
    p->d_ops.push_back(o);
    p->d_mats.push_back(t);
  }
  return CCUT_OK;
}

hipError_t pin_begin(ccut_ctx *c);

ccut_status check_eval(ccut_plan *p, const ccut_eval_opts *eo) {
  if (!p || !eo) return CCUT_E_INVALID;
  ccut_ctx *c = p->ctx;
  if (eo->precision != CCUT_FP64 && eo->precision != CCUT_FP32_MFMA_FP64SUM &&
      eo->precision != CCUT_FP32X3_MFMA_FP64SUM)
    return fail(c, CCUT_E_INVALID, "unknown precision mode");
  if (eo->method > CCUT_METHOD_HEISENBERG) return fail(c, CCUT_E_INVALID, "unknown evaluation method");
  if (eo->flags & ~(uint32_t)(CCUT_FLAG_SPARSE | CCUT_FLAG_SETTLE | CCUT_FLAG_ML | CCUT_FLAG_SKIP))
    return fail(c, CCUT_E_INVALID, "unknown evaluation flag");
  // shot counters and histogram counts are 32-bit per variant
  if (eo->shots_per_variant > 0xFFFFFFFFull)
    return fail(c, CCUT_E_INVALID, "shots_per_variant must be below 2^32");
  if (c->device < 0) return fail(c, CCUT_E_DEVICE, "host-only context: evaluation needs a device");
  HIP_TRY(c, hipSetDevice(c->device));
  c->cancel.store(0);
  c->arena.reset();
  c->staged.clear();
  c->call_upload_bytes = 0;
  if (!c->capturing) HIP_TRY(c, pin_begin(c));
  if (!c->aux) {
    HIP_TRY(c, hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking));
    HIP_TRY(c, hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming));
    HIP_TRY(c, hipEventCreateWithFlags(&c->join_ev, hipEventDisableTiming));
  }
  c->cur = c->stream;
  // the auxiliary stream starts after everything already queued on the caller's stream
  HIP_TRY(c, hipEventRecord(c->fork_ev, c->stream));
  HIP_TRY(c, hipStreamWaitEvent(c->aux, c->fork_ev, 0));
  return ensure_ops(p);
}

// Route the next launches of fragment f: non-Clifford fragments go to the
// auxiliary stream so they overlap the Clifford chain.
void route(ccut_ctx *c, const Fragment &f) { c->cur = (f.clifford || !c->use_aux) ? c->stream : c->aux; }

// Join the auxiliary stream back into the caller's stream.
ccut_status join(ccut_ctx *c) {
  c->cur = c->stream;
  if (!c->use_aux) return CCUT_OK;
  HIP_TRY(c, hipEventRecord(c->join_ev, c->aux));
  HIP_TRY(c, hipStreamWaitEvent(c->stream, c->join_ev, 0));
  return CCUT_OK;
}

// Start a call's staging slot: mark the previous slot's work with events on
// both streams, move to the next slot and wait until its last use is done.
hipError_t pin_begin(ccut_ctx *c) {
  if (c->pin_cur >= 0) {
    ccut_ctx::PinSlot &prev = c->pin[c->pin_cur];
    if (!prev.ev_s) {
      hipError_t e = hipEventCreateWithFlags(&prev.ev_s, hipEventDisableTiming);
      if (e != hipSuccess) return e;
      if ((e = hipEventCreateWithFlags(&prev.ev_a, hipEventDisableTiming)) != hipSuccess) return e;
    }
    hipError_t e = hipEventRecord(prev.ev_s, c->stream);
    if (e != hipSuccess) return e;
    if (c->aux && (e = hipEventRecord(prev.ev_a, c->aux)) != hipSuccess) return e;
    prev.pending = true;
  }
  c->pin_cur = (c->pin_cur + 1) % ccut_ctx::kPinSlots;
  ccut_ctx::PinSlot &sl = c->pin[c->pin_cur];
  if (sl.pending) {
    hipError_t e = hipEventSynchronize(sl.ev_s);
    if (e != hipSuccess) return e;
    if (c->aux && (e = hipEventSynchronize(sl.ev_a)) != hipSuccess) return e;
    sl.pending = false;
  }
  sl.chunk = 0;
  sl.used = 0;
  return hipSuccess;
}

// Copy host bytes to fresh device memory on the current stream, staged in
// the call's pinned slot.  A null source (an empty host vector) gets the
// allocation without a copy.
void *upload(ccut_ctx *c, const void *src, size_t bytes) {
  const size_t need = (bytes + 255) & ~size_t(255);
  if (CallGraph *g = c->capturing; g && src && bytes) {
    // kept for good in the captured call's device block; its one copy is
    // enqueued after the capture ends, ahead of the first launch
    if (g->pin_used + need > g->pin_cap) return nullptr;
    std::memcpy(g->pin + g->pin_used, src, bytes);
    void *d = g->dev + g->pin_used;
    g->pin_used += need;
    c->call_upload_bytes += need;
    return d;
  }
  void *d = c->arena.get(bytes);
  if (!d) return nullptr;
  if (!src || bytes == 0) return d;
  // a multiply-xorshift hash of the bytes, eight at a time
  uint64_t hsh = 0x9E3779B97F4A7C15ull ^ bytes;
  {
    const unsigned char *q = static_cast<const unsigned char *>(src);
    size_t i = 0;
    for (; i + 8 <= bytes; i += 8) {
      uint64_t w;
      std::memcpy(&w, q + i, 8);
      hsh = (hsh ^ w) * 0xFF51AFD7ED558CCDull;
      hsh ^= hsh >> 29;
    }
    for (; i < bytes; ++i) hsh = (hsh ^ q[i]) * 0xC4CEB9FE1A85EC53ull;
  }
  Arena &A = c->arena;
  const size_t ui = A.n_uploads++;
  if (c->replay_uploads) {
    // replay: the bytes are already there, provided this is the same upload
    // as in the run that copied them
    if (ui < A.upload_hash.size() && A.upload_hash[ui] == hsh) return d;
    return nullptr;  // (a re-enqueue that does not repeat the first one's uploads)
  }
  if (A.upload_hash.size() <= ui) A.upload_hash.resize(ui + 1);
  A.upload_hash[ui] = hsh;
  c->call_upload_bytes += need;
  if (c->pin_cur < 0 && pin_begin(c) != hipSuccess) return nullptr;
  ccut_ctx::PinSlot &sl = c->pin[c->pin_cur];
  while (sl.chunk < sl.chunks.size() && sl.used + need > sl.chunks[sl.chunk].second) {
    ++sl.chunk;
    sl.used = 0;
  }
  if (sl.chunk == sl.chunks.size()) {
    const size_t cap = std::max<size_t>(need, size_t(1) << 20);
    char *h = nullptr;
    if (hipHostMalloc((void **)&h, cap, hipHostMallocDefault) != hipSuccess) return nullptr;
    sl.chunks.push_back({h, cap});
    sl.used = 0;
  }
  char *stage = sl.chunks[sl.chunk].first + sl.used;
  sl.used += need;
  std::memcpy(stage, src, bytes);
  if (hipMemcpyAsync(d, stage, bytes, hipMemcpyHostToDevice, c->cur) != hipSuccess) return nullptr;
  return d;
}

uint32_t row_words(uint32_t m) {
  const uint32_t w = (m + 63) / 64;
  return w <= 1 ? 1 : w <= 2 ? 2 : w <= 4 ? 4 : w <= 8 ? 8 : 0;
}

ccut_status check_request(ccut_ctx *c, uint32_t n, const uint32_t *qubits, uint32_t nq,
                          uint32_t max_nq = 24) {
  if (nq > max_nq) return fail(c, CCUT_E_INVALID, "marginal over more than 24 qubits");
  if (nq && !qubits) return fail(c, CCUT_E_INVALID, "qubits is NULL");
  std::vector<char> seen(n, 0);
  for (uint32_t i = 0; i < nq; ++i) {
    if (qubits[i] >= n) return fail(c, CCUT_E_INVALID, "requested qubit out of range");
    if (seen[qubits[i]]) return fail(c, CCUT_E_INVALID, "requested qubit repeated");
    seen[qubits[i]] = 1;
  }
  return CCUT_OK;
}

ccut_status cancelled(ccut_ctx *c) {
  if (c->cancel.load()) return fail(c, CCUT_E_CANCELLED, "cancelled");
  return CCUT_OK;
}

FragDev frag_desc(ccut_plan *p, const Fragment &f, const FragRequest &r, uint32_t circuit) {
  FragDev h = make_frag_dev(f, r, ((uint64_t)circuit << 40) | ((uint64_t)f.index << 32));
  h.ops = p->d_ops[f.index];
  h.mats = p->d_mats[f.index];
  h.layers = p->d_layers[f.index];
  h.n_layers = p->n_layers[f.index];
  return h;
}

// The measured Paulis of a Clifford fragment before the pull-back through
// its gates, in measured order: a requested output's Z, a quantum output's X
// then Z (its basis Pauli is X, Z or i X Z); rows x[W], z[W], sign word.
std::vector<uint64_t> measured_rows(const FragDev &h, uint32_t W) {
  const uint32_t RW = 2 * W + 1;
  std::vector<uint64_t> rows;
  auto add = [&](bool xpart, uint32_t q) {
    std::vector<uint64_t> row(RW, 0);
    row[(xpart ? 0 : W) + (q >> 6)] = 1ull << (q & 63);
    rows.insert(rows.end(), row.begin(), row.end());
  };
  for (uint32_t j = 0; j < h.n_meas; ++j) {
    const uint32_t q = h.meas[j];
    bool out = false;
    for (uint32_t a = 0; a < h.n_axes; ++a) out |= h.axis_side[a] == 0 && h.axis_local[a] == q;
    if (out) add(true, q);
    add(false, q);
  }
  return rows;
}

// Affine sample models of variants [v0, v0 + nv) of a Clifford fragment:
// its measured Paulis are carried back through the fragment once (the
// reversed stream of inverse gates), then one wave per variant eliminates
// them against the variant's prepared product state (Heisenberg picture).
// The same rows for a measured set of any size (meas: local qubits in
// measured order); row_of[j] = the first row of measurement j, meas_axis[j]
// = the axis of a quantum output, else -1.
std::vector<uint64_t> measured_rows(const Fragment &f, const std::vector<uint32_t> &meas, uint32_t W,
                                    std::vector<uint16_t> *row_of = nullptr, std::vector<int8_t> *meas_axis = nullptr) {
  const uint32_t RW = 2 * W + 1;
  std::vector<uint64_t> rows;
  auto add = [&](bool xpart, uint32_t q) {
    std::vector<uint64_t> row(RW, 0);
    row[(xpart ? 0 : W) + (q >> 6)] = 1ull << (q & 63);
    rows.insert(rows.end(), row.begin(), row.end());
  };
  for (uint32_t q : meas) {
    int axis = -1;
    for (size_t a = 0; a < f.axes.size(); ++a)
      if (f.axes[a].side == 0 && f.axes[a].local == q) axis = (int)a;
    if (row_of) row_of->push_back((uint16_t)(rows.size() / RW));
    if (meas_axis) meas_axis->push_back((int8_t)axis);
    if (axis >= 0) add(true, q);
    add(false, q);
  }
  return rows;
}

// vmask (device, one byte per variant of the fragment, optional): variants
// with vmask[v] == 0 get no model (64 measured qubits or fewer; wider
// fragments model every variant)
ccut_status tableau_models(ccut_plan *p, const Fragment &f, const FragDev &h, const FragRequest &r, uint64_t v0,
                           uint64_t nv, uint64_t *models, const uint8_t *vmask = nullptr) {
  ccut_ctx *c = p->ctx;
  const uint32_t W = row_words(f.m());
  if (!W) return fail(c, CCUT_E_UNSUPPORTED, "Clifford fragment wider than 512 qubits");
  const uint32_t nm = (uint32_t)r.meas.size();
  if (nm > (uint32_t)kMaxMeasWide) return fail(c, CCUT_E_UNSUPPORTED, "more than 1024 measured qubits in a fragment");
  std::vector<uint16_t> row_of;
  std::vector<int8_t> meas_axis;
  std::vector<uint64_t> rows = measured_rows(f, r.meas, W, &row_of, &meas_axis);
  const uint32_t n_rows = (uint32_t)(rows.size() / (2 * W + 1));
  if (rows.empty()) rows.assign(2 * W + 1, 0);  // nothing measured: a valid buffer all the same
  uint64_t *d_in = (uint64_t *)upload(c, rows.data(), rows.size() * 8);
  uint64_t *d_out = aget<uint64_t>(c, rows.size());
  if (!d_in || !d_out) return fail(c, CCUT_E_OOM, "device allocation failed");
  FragDev hb = h;
  hb.ops = p->d_back[f.index];
  hb.n_ops = p->n_back[f.index];
  hb.layers = p->d_back_layers[f.index];
  hb.n_layers = p->n_back_layers[f.index];
  int8_t *d_axis = nullptr;
  uint16_t *d_row = nullptr;
  if (nm > (uint32_t)kMaxMeas) {
    d_axis = (int8_t *)upload(c, meas_axis.data(), meas_axis.size());
    d_row = (uint16_t *)upload(c, row_of.data(), row_of.size() * 2);
    if (!d_axis || !d_row) return fail(c, CCUT_E_OOM, "device allocation failed");
  }
  KTimer t(c, CCUT_K_AFFINE);
  HIP_TRY(c, launch_rows(hb, W, d_in, d_out, n_rows, c->cur));
  if (nm > (uint32_t)kMaxMeas)
    HIP_TRY(c, launch_affine_wide(h, W, d_axis, d_row, nm, d_out, v0, nv, models, c->cur));
  else
    HIP_TRY(c, launch_affine(h, W, d_out, v0, nv, models, c->cur, vmask));
  return CCUT_OK;
}

// Per-variant outcome distributions dist[v][x] over the measured set.
// cnt_out (sampled Clifford fragments, fewer than 2^16 shots): the tables
// as 16-bit shot counts into *cnt_out instead (*dist_out null).
// Maximum-likelihood correction of a fragment's variant tables, in place
// (Sec. V-C, distribution builder; launch_ml_correct).  Fragments without
// quantum outputs keep their tables: sampled histograms already are
// physical models.
ccut_status ml_correct(ccut_ctx *c, const Fragment &f, const FragRequest &r, double *dist) {
  MlJob J{};
  uint64_t stride = 1;
  for (size_t j = 0; j < f.axes.size(); ++j) {
    if (f.axes[j].side == 0) {
      if (J.n_out == kMlMaxOut)
        return fail(c, CCUT_E_UNSUPPORTED, "maximum-likelihood correction of more than 2 quantum outputs");
      J.opos[J.n_out] = (uint32_t)r.axis_outpos[j];
      J.ostride[J.n_out++] = (uint32_t)stride;
    } else {
      J.istride[J.n_in++] = (uint32_t)stride;
    }
    stride *= f.axes[j].radix();
  }
  if (J.n_out == 0) return CCUT_OK;
  if (J.n_in > 8) return fail(c, CCUT_E_UNSUPPORTED, "maximum-likelihood correction of more than 8 quantum inputs");
  J.n_req = (uint32_t)r.req_pos.size();
  for (uint32_t i = 0; i < J.n_req; ++i) J.xpos[i] = r.req_pos[i];
  J.dist = dist;
  J.nx = 1ull << J.n_req;
  J.row_len = 1ull << r.meas.size();
  J.n_prep = 1u << (2 * J.n_in);
  J.eig = aget<double>(c, (size_t)J.n_prep * J.nx << J.n_out);
  J.tau = aget<double>(c, J.n_prep);
  MlJob *d = (MlJob *)upload(c, &J, sizeof(MlJob));
  if (!J.eig || !J.tau || !d) return fail(c, CCUT_E_OOM, "device allocation failed");
  KTimer t(c, CCUT_K_TRANSFORM);
  HIP_TRY(c, launch_ml_correct(J, d, c->cur));
  return CCUT_OK;
}

// vmask (device, one byte per variant, optional): sampled Clifford variants
// with vmask[v] == 0 draw no shots (all-zero tables)
ccut_status variant_dists(ccut_plan *p, const ccut_eval_opts *eo, const Fragment &f,
                          const FragRequest &r, double **dist_out, uint64_t *pre_models = nullptr,
                          uint16_t **cnt_out = nullptr, const uint8_t *vmask = nullptr) {
  ccut_ctx *c = p->ctx;
  const uint32_t nm = (uint32_t)r.meas.size();
  const uint64_t nv = f.n_variants;
  if (f.clifford && nm > (uint32_t)kMaxMeas)
    return fail(c, CCUT_E_UNSUPPORTED, "Clifford fragment with more than 64 measured qubits");
  if (nm > (uint32_t)kMaxTableBits)
    return fail(c, CCUT_E_UNSUPPORTED, "outcome table over more than 24 measured qubits");
  if ((nv << nm) > (uint64_t(1) << 34))
    return fail(c, CCUT_E_UNSUPPORTED, "variant tables exceed 2^34 entries");
  const FragDev h = frag_desc(p, f, r, eo->circuit);
  const bool want16 = cnt_out && f.clifford && eo->shots_per_variant > 0 && eo->shots_per_variant <= 0xFFFFull;
  uint16_t *cnt16 = want16 ? aget<uint16_t>(c, nv << nm) : nullptr;
  double *dist = want16 ? nullptr : aget<double>(c, nv << nm);
  if (!dist && !cnt16) return fail(c, CCUT_E_OOM, "device allocation failed");
  if (cnt_out) *cnt_out = cnt16;
  if (!f.clifford) {
    const size_t sb = sv_states_bytes(h);
    double *states = sb ? aget<double>(c, sb / sizeof(double)) : nullptr;
    if (sb && !states) return fail(c, CCUT_E_OOM, "device allocation failed");
    KTimer t(c, CCUT_K_SV);
    HIP_TRY(c, launch_sv(h, dist, states, c->cur));
  } else {
    uint64_t *models = pre_models;
    if (!models) {
      models = aget<uint64_t>(c, nv * model_words(nm));
      if (!models) return fail(c, CCUT_E_OOM, "device allocation failed");
      // (exact tables read every model: only sampled data skip some)
      ccut_status st2 = tableau_models(p, f, h, r, 0, nv, models, eo->shots_per_variant ? vmask : nullptr);
      if (st2 != CCUT_OK) return st2;
    }
    if (eo->shots_per_variant == 0) {
      KTimer t(c, CCUT_K_EXACT);
      HIP_TRY(c, launch_exact_tables(models, nm, nv, dist, c->cur));
    } else {
      const uint64_t shots = eo->shots_per_variant;
      const uint32_t bins = 1u << nm;
      const uint64_t nquads = (shots + 3) / 4;
      for (uint64_t v0 = 0; v0 < nv; v0 += 65535) {
        const uint64_t cnv = std::min<uint64_t>(65535, nv - v0);
        const bool lds = nm <= kLdsHistBits;
        uint32_t nblk = 1;
        if (lds) {
          // enough shots per workgroup that its partial histogram is not mostly
          // empty, few enough for its 16-bit LDS counts
          const uint64_t per_block = std::max<uint64_t>(bins, 2048);
          uint64_t want = (shots + per_block - 1) / per_block;
          uint64_t maxb = (nquads + kSampleThreads - 1) / kSampleThreads;
          nblk = (uint32_t)std::max<uint64_t>(1, std::min(want, maxb));
          nblk = (uint32_t)std::max<uint64_t>(nblk, (nquads + kMaxUnitQpt * kSampleThreads - 1) / (kMaxUnitQpt * kSampleThreads));
        } else {
          nblk = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((nquads + 1023) / 1024, 4096));
        }
        const uint32_t qpt = (uint32_t)((nquads + (uint64_t)nblk * kSampleThreads - 1) / ((uint64_t)nblk * kSampleThreads));
        const uint64_t pcount = lds ? cnv * nblk * (uint64_t)bins : cnv * (uint64_t)bins;
        uint32_t *partial = aget<uint32_t>(c, pcount);
        if (!partial) return fail(c, CCUT_E_OOM, "device allocation failed");
        if (!lds) HIP_TRY(c, launch_fill_u32(partial, pcount, 0u, c->cur));
        {
          KTimer t(c, CCUT_K_SAMPLE);
          HIP_TRY(c, launch_sample_hist(models + v0 * model_words(nm), nm, cnv, shots, eo->seed,
                                        h.vid_base + v0, partial, nblk, qpt, nullptr, c->cur,
                                        vmask ? vmask + v0 : nullptr));
        }
        {
          KTimer t(c, CCUT_K_HIST_REDUCE);
          HIP_TRY(c, launch_hist_reduce(partial, cnv, lds ? nblk : 1, bins, shots, dist ? dist + (v0 << nm) : nullptr,
                                        c->cur, cnt16 ? cnt16 + (v0 << nm) : nullptr));
        }
      }
    }
  }
  *dist_out = dist;
  if ((eo->flags & CCUT_FLAG_ML) && dist) {
    ccut_status st = ml_correct(c, f, r, dist);
    if (st != CCUT_OK) return st;
  }
  return cancelled(c);
}

// Per-axis Pauli-basis passes: data[v][x] -> T[p_f][rest], where rest is
// the x part with the output bits removed (mode 1) or the J part consumed
// (mode 2, parity tables laid out [v][J][string]).
// Tile plan of a fragment's marginal-mode transform (variant data in, T out):
// false when the fragment has no axes, more than kMaxTileAxes, or variant
// data per x_out entry beyond kTileElems.
bool tile_job(const Fragment &f, const FragRequest &r, const double *in, uint64_t xsize, double *out, TileJob &J) {
  const uint32_t a = (uint32_t)f.axes.size();
  if (a == 0 || a > (uint32_t)kMaxTileAxes) return false;
  J = TileJob{};
  uint64_t V = 1;
  uint32_t n_out = 0;
  std::vector<uint32_t> outpos;
  for (uint32_t j = 0; j < a; ++j) {
    const bool is_out = f.axes[j].side == 0;
    J.rad[j] = is_out ? 3u : 4u;
    V *= J.rad[j];
    if (is_out) {
      ++n_out;
      outpos.push_back((uint32_t)r.axis_outpos[j]);
    }
  }
  if ((V << n_out) > kTileElems) return false;
  uint32_t xb = 0;  // log2 of x_in
  while ((1ull << xb) < xsize) ++xb;
  const uint32_t xo_bits = xb - n_out;
  uint32_t t = std::min<uint32_t>(xo_bits, kTileMaxT);
  while ((V << (n_out + t)) > kTileElems) --t;
  std::sort(outpos.begin(), outpos.end());
  auto is_out_pos = [&](uint32_t p) { return std::binary_search(outpos.begin(), outpos.end(), p); };
  uint32_t p = 0, cnt = 0;
  while (cnt < t) {
    if (!is_out_pos(p)) J.xpos[cnt++] = p;
    ++p;
  }
  const uint32_t thr = p;
  uint32_t nh = 0;
  for (uint32_t q : outpos)
    if (q >= thr) J.hpos[nh++] = q;
  for (uint32_t j = 0; j < a; ++j) {
    if (J.rad[j] != 3) continue;
    const uint32_t q = (uint32_t)r.axis_outpos[j];
    uint32_t lp = q;
    if (q >= thr) {
      lp = thr;
      while (J.hpos[lp - thr] != q) ++lp;
    }
    J.lpos[j] = lp;
  }
  uint64_t Rj = 1;
  for (uint32_t j = 0; j < a; ++j) {
    J.rmag[j] = Rj == 1 ? 0u : (uint32_t)((1ull << 32) / Rj + 1);
    Rj *= J.rad[j];
  }
  J.in = in;
  J.out = out;
  J.x_in = xsize;
  J.x_out = xsize >> n_out;
  J.tiles = (uint32_t)(J.x_out >> t);
  J.n_axes = a;
  J.v_count = (uint32_t)V;
  J.t = t;
  J.thr = thr;
  J.nh = nh;
  J.lbits = thr + nh;
  return true;
}

ccut_status pauli_passes(ccut_ctx *c, const Fragment &f, const FragRequest &r, double *data,
                         uint64_t xsize, uint64_t mode2_lo, double **out) {
  const uint32_t a = (uint32_t)f.axes.size();
  if (!mode2_lo && a) {
    // every axis in one launch, through LDS tiles (the passes' arithmetic)
    TileJob J;
    if (tile_job(f, r, data, xsize, nullptr, J)) {
      J.out = aget<double>(c, J.x_out << (2 * a));
      TileJob *dj = J.out ? (TileJob *)upload(c, &J, sizeof(J)) : nullptr;
      if (!dj) return fail(c, CCUT_E_OOM, "device allocation failed");
      KTimer t(c, CCUT_K_TRANSFORM);
      HIP_TRY(c, launch_transform_tiled(dj, 1, J.tiles, c->cur));
      *out = J.out;
      return CCUT_OK;
    }
  }
  // String-selection tables that are small (up to 3 axes, at most 27 terms
  // per entry, at most 2^16 entries out) take all axes in one launch: there
  // the launches, not the arithmetic, are the cost; the rest take the
  // per-axis passes, which read each entry a bounded number of times.
  uint64_t n_out_axes = 0;
  for (const Axis &ax : f.axes) n_out_axes += ax.side == 0;
  const uint64_t entries_out = (mode2_lo ? mode2_lo : xsize >> n_out_axes) << (2 * a);
  if (mode2_lo && a >= 2 && a <= 3 && entries_out <= (1ull << 16)) {
    TransformAll A{};
    A.n_axes = a;
    A.x_in = xsize;
    A.n_strings = mode2_lo;
    uint64_t xo = xsize, nout = 0;
    for (uint32_t j = 0; j < a; ++j) {
      const bool is_out = f.axes[j].side == 0;
      A.rad[j] = f.axes[j].radix();
      A.mode[j] = is_out ? (mode2_lo ? 2u : 1u) : 0u;
      A.pos[j] = is_out && !mode2_lo ? (uint32_t)r.axis_outpos[j] : 0u;
      if (is_out) ++nout;
    }
    xo >>= nout;
    if (mode2_lo) xo = mode2_lo;
    A.x_out = xo;
    double *nxt = aget<double>(c, xo << (2 * a));
    if (!nxt) return fail(c, CCUT_E_OOM, "device allocation failed");
    {
      KTimer t(c, CCUT_K_TRANSFORM);
      HIP_TRY(c, launch_transform_all(A, data, nxt, c->cur));
    }
    *out = nxt;
    return CCUT_OK;
  }
  std::vector<uint64_t> rad(a);
  for (uint32_t j = 0; j < a; ++j) rad[j] = f.axes[j].radix();
  std::vector<int32_t> pos(r.axis_outpos.begin(), r.axis_outpos.end());
  double *cur = data;
  for (uint32_t j = 0; j < a; ++j) {
    uint64_t outer = 1, R = 1;
    for (uint32_t l = j + 1; l < a; ++l) outer *= rad[l];
    for (uint32_t l = 0; l < j; ++l) R *= rad[l];
    const bool is_out = f.axes[j].side == 0;
    const uint64_t xout = is_out ? xsize / 2 : xsize;
    double *nxt = aget<double>(c, outer * 4 * R * xout);
    if (!nxt) return fail(c, CCUT_E_OOM, "device allocation failed");
    int mode = 0;
    uint64_t lo = 1;
    if (is_out) {
      if (mode2_lo) {
        mode = 2;
        lo = mode2_lo;
      } else {
        mode = 1;
        lo = 1ull << pos[j];
        for (uint32_t l = j + 1; l < a; ++l)
          if (pos[l] > pos[j]) pos[l] -= 1;
      }
    }
    {
      KTimer t(c, CCUT_K_TRANSFORM);
      HIP_TRY(c, launch_transform_pass(cur, nxt, outer, R, xsize, lo, mode, c->cur));
    }
    cur = nxt;
    rad[j] = 4;
    xsize = xout;
  }
  *out = cur;
  return CCUT_OK;
}


// Exact Pauli-basis tensor of a Clifford fragment in the Heisenberg picture.
// Marginal mode (strings == nullptr): T[p_f][b] over the requested outputs.
// String mode: t[p_f][s] for Z strings given as local z masks (W words each).
ccut_status heis_tensor(ccut_plan *p, const Fragment &f, const FragRequest &r, uint32_t circuit,
                        const std::vector<std::vector<uint64_t>> *strings, double **out) {
  ccut_ctx *c = p->ctx;
  const uint32_t W = row_words(f.m());
  if (!W) return fail(c, CCUT_E_UNSUPPORTED, "Clifford fragment wider than 512 qubits");
  const uint32_t RW = 2 * W + 1;
  std::vector<uint64_t> rows;
  auto add_row = [&](int xq, int zq, const std::vector<uint64_t> *zmask) {
    std::vector<uint64_t> row(RW, 0);
    if (xq >= 0) row[xq >> 6] |= 1ull << (xq & 63);
    if (zq >= 0) row[W + (zq >> 6)] |= 1ull << (zq & 63);
    if (zmask)
      for (uint32_t w = 0; w < W; ++w) row[W + w] |= (*zmask)[w];
    rows.insert(rows.end(), row.begin(), row.end());
  };
  const uint32_t nreq = (uint32_t)r.req_pos.size();
  if (!strings) {
    for (uint32_t i = 0; i < nreq; ++i) add_row(-1, (int)r.meas[r.req_pos[i]], nullptr);
  } else {
    for (const auto &z : *strings) add_row(-1, -1, &z);
  }
  uint32_t n_in = 0, n_out = 0;
  for (const Axis &a : f.axes) {
    if (a.side == 0) {
      add_row((int)a.local, -1, nullptr);
      add_row(-1, (int)a.local, nullptr);
      ++n_out;
    } else {
      ++n_in;
    }
  }
  if (n_out > 8) return fail(c, CCUT_E_UNSUPPORTED, "more than 8 quantum outputs on a Clifford fragment");
  std::vector<uint64_t> cin(8, 0);
  for (uint32_t i = 0; i < f.m(); ++i)
    if (f.segs[i] == 0) cin[i >> 6] |= 1ull << (i & 63);
  const uint32_t n_rows = (uint32_t)(rows.size() / RW);
  if (rows.empty()) rows.assign(RW, 0);  // a fragment with nothing to carry back still gets a valid buffer
  const uint64_t ncols = strings ? strings->size() : (1ull << nreq);
  const uint64_t total = ncols << (2 * f.axes.size());
  if (total > (1ull << 34)) return fail(c, CCUT_E_UNSUPPORTED, "Pauli-basis tensor exceeds 2^34 entries");
  double *tau = aget<double>(c, total);
  uint64_t *d_out = aget<uint64_t>(c, rows.size());
  uint64_t *d_in = (uint64_t *)upload(c, rows.data(), rows.size() * 8);
  if (!tau || !d_out || !d_in) return fail(c, CCUT_E_OOM, "device allocation failed");
  FragRequest rq = r;
  FragDev h = frag_desc(p, f, rq, circuit);
  h.ops = p->d_back[f.index];  // the carry-back stream
  h.n_ops = p->n_back[f.index];
  h.layers = p->d_back_layers[f.index];
  h.n_layers = p->n_back_layers[f.index];
  {
    KTimer t(c, CCUT_K_HEISENBERG);
    HIP_TRY(c, launch_heisenberg(h, W, n_in, n_out, strings ? 0 : nreq, strings ? (uint32_t)strings->size() : 0,
                                 cin.data(), d_in, d_out, n_rows, tau, c->cur));
  }
  *out = tau;
  return cancelled(c);
}


// Operands of the dense contraction: the fragment with the most requested
// bits forms the column side, the others the row side.
void make_gemm_args(const RecombArgs &args, GemmArgs &g) {
  g = GemmArgs{};
  g.k = args.k;
  g.K = 1ull << (2 * args.k);
  g.lo_parts = args.lo_parts;
  uint32_t rf = 0;
  for (uint32_t f = 1; f < args.n_frags; ++f)
    if (args.f[f].n_req > args.f[rf].n_req) rf = f;
  uint32_t lbits = 0;
  for (uint32_t f = 0; f < args.n_frags; ++f) {
    g.f[f] = args.f[f];
    bool ident = args.f[f].n_axes == args.k;
    for (uint32_t j = 0; ident && j < args.f[f].n_axes; ++j) ident = args.f[f].axis_cut[j] == j;
    g.ident[f] = ident ? 1u : 0u;
    GemmSide &S = (f == rf) ? g.R : g.L;
    const uint32_t sh = (f == rf) ? 0u : lbits;
    S.frag[S.n] = f;
    S.shift[S.n] = sh;
    S.bits[S.n] = args.f[f].n_req;
    S.n++;
    if (f != rf) lbits += args.f[f].n_req;
  }
  g.M = 1u << lbits;
  g.N = 1u << args.f[rf].n_req;
}

// allow_skinny: exhaustive contractions with at most 32 rows take the
// skinny kernel (term-list estimates always take the MFMA tiles)
ccut_status run_gemm(ccut_ctx *c, const GemmArgs &g, bool fp32, double *res, bool allow_skinny = false) {
  const bool skinny = allow_skinny && contraction_skinny(g, fp32);
  const uint32_t splits = contraction_splits(g, skinny);
  GemmArgs *dg = (GemmArgs *)upload(c, &g, sizeof(g));
  double *partial = aget<double>(c, (size_t)splits * g.M * g.N);
  if (!dg || !partial) return fail(c, CCUT_E_OOM, "device allocation failed");
  KTimer t(c, CCUT_K_RECOMBINE);
  HIP_TRY(c, launch_recombine_gemm(g, dg, fp32, partial, splits, res, c->cur, skinny));
  return CCUT_OK;
}

// The sparse contraction: the support (cut terms whose column is nonzero in
// every fragment) is found on the device, its size read back, and only its
// terms are summed: the plain sum in ascending order when it is small (the
// same operations as the dense plain sum minus its zero terms), else the
// term-list contraction.
// The contraction over a term list (device, ascending, count terms): the
// plain fp64 sum over the terms when small, else the matrix paths.
ccut_status contract_terms(ccut_ctx *c, const RecombArgs &args, const RecombArgs *dargs, uint32_t nq, bool fp32,
                           double *res, const uint64_t *terms, uint64_t count) {
  if (count == 0) {  // every term vanishes
    HIP_TRY(c, launch_fill_u32(reinterpret_cast<uint32_t *>(res), 2ull << nq, 0u, c->cur));  // +0.0
    return CCUT_OK;
  }
  if (!fp32 && (count << nq) <= (1ull << 20) && args.n_frags <= 8) {
    KTimer t(c, CCUT_K_RECOMBINE);
    HIP_TRY(c, launch_recombine_terms(dargs, nq, terms, count, res, c->cur));
    return CCUT_OK;
  }
  GemmArgs g;
  make_gemm_args(args, g);
  g.terms = terms;
  g.K = count;
  return run_gemm(c, g, fp32, res, true);
}

ccut_status recombine_sparse(ccut_ctx *c, const RecombArgs &args, uint32_t nq, bool fp32, double *res) {
  const uint64_t K = 1ull << (2 * args.k);
  SupportArgs sa{};
  uint64_t cols_total = 0;
  for (uint32_t f = 0; f < args.n_frags; ++f) {
    sa.off[f] = cols_total;
    cols_total += 1ull << (2 * args.f[f].n_axes);
  }
  RecombArgs *dargs = (RecombArgs *)upload(c, &args, sizeof(args));
  uint8_t *nz = aget<uint8_t>(c, cols_total);
  uint64_t *pos = aget<uint64_t>(c, K), *scratch = aget<uint64_t>(c, scan_scratch_words(K));
  uint64_t *terms = aget<uint64_t>(c, K);
  if (!dargs || !nz || !pos || !scratch || !terms) return fail(c, CCUT_E_OOM, "device allocation failed");
  uint64_t count = 0;
  {
    KTimer t(c, CCUT_K_RECOMBINE);
    for (uint32_t f = 0; f < args.n_frags; ++f)
      HIP_TRY(c, launch_colnz(args.f[f].T, args.f[f].rows, 1ull << (2 * args.f[f].n_axes), nz + sa.off[f], c->cur));
    HIP_TRY(c, launch_support_terms(dargs, sa, nz, K, pos, scratch, terms, c->cur));
  }
  HIP_TRY(c, hipMemcpyAsync(&count, pos + K - 1, 8, hipMemcpyDeviceToHost, c->cur));
  HIP_TRY(c, hipStreamSynchronize(c->cur));
  return contract_terms(c, args, dargs, nq, fp32, res, terms, count);
}

// Contract the fragment tensors into out[2^nq].  fp64 with at most 2^20
// term-outputs: the plain ascending sum; otherwise the K-split MFMA contraction
// (fp32 products with fp64 across K-chunks, or fp64 MFMA).
// The plain fp64 sum (per output, every term's product, ascending) for
// small contractions of more than two fragments; two fragments always take
// the matrix paths (the skinny kernel's ascending sum of products is the
// plain sum's arithmetic, and it streams the column tensor).
bool plain_contraction(const RecombArgs &args, uint32_t nq, bool fp32) {
  const uint64_t K = 1ull << (2 * args.k);
  return !fp32 && args.n_frags > 2 && (K << nq) <= (1ull << 20);
}

ccut_status recombine(ccut_ctx *c, const RecombArgs &args, uint32_t nq, bool fp32, double *res,
                      bool sparse = false) {
  if (sparse) return recombine_sparse(c, args, nq, fp32, res);
  const uint64_t K = 1ull << (2 * args.k);
  if (plain_contraction(args, nq, fp32)) {
    RecombArgs *dargs = (RecombArgs *)upload(c, &args, sizeof(args));
    if (!dargs) return fail(c, CCUT_E_OOM, "device allocation failed");
    KTimer t(c, CCUT_K_RECOMBINE);
    HIP_TRY(c, launch_recombine_fp64(dargs, args.n_frags, nq, res, c->cur));
    return CCUT_OK;
  }
  GemmArgs g;
  make_gemm_args(args, g);
  return run_gemm(c, g, fp32, res, true);
}

// Exact-mode Clifford fragments take the Heisenberg picture unless told
// otherwise; a marginal request of more than 14 bits on the fragment
// (req_bits) takes the variant path, since the transform to the Pauli basis
// runs one LDS block of 2^req_bits entries per row (Z strings: req_bits 0).
constexpr uint32_t kHeisMaxReqBits = 14;
bool use_heisenberg(const Fragment &f, const ccut_eval_opts *eo, size_t req_bits) {
  return f.clifford && eo->shots_per_variant == 0 && eo->method != CCUT_METHOD_VARIANTS &&
         req_bits <= kHeisMaxReqBits;
}

// Results to the caller: into host memory with a final synchronization, or
// into device memory in stream order (the copy is the call's last work on
// the context's stream; no synchronization).
ccut_status finish_out(ccut_ctx *c, const double *dev, double *out, size_t count, int on_device) {
  HIP_TRY(c, hipMemcpyAsync(out, dev, count * sizeof(double),
                            on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->cur));
  if (!on_device) HIP_TRY(c, hipStreamSynchronize(c->cur));
  return CCUT_OK;
}

}  // namespace

// ====================================================================== ABI

extern "C" {

ccut_status ccut_ctx_create(const ccut_opts *opts, ccut_ctx **out) {
  g_create_err.clear();
  if (!out) return CCUT_E_INVALID;
  *out = nullptr;
  std::unique_ptr<ccut_ctx> c(new (std::nothrow) ccut_ctx());
  if (!c) return CCUT_E_OOM;
  ccut_opts o{};
  if (opts) o = *opts;
  c->device = opts ? o.device : 0;
  c->stream = (hipStream_t)o.hip_stream;
  c->arena.alloc = o.alloc;
  c->arena.free_fn = o.free;
  c->arena.user = o.user;
  if ((o.alloc == nullptr) != (o.free == nullptr)) {
    g_create_err = "alloc and free must both be set or both be NULL";
    return CCUT_E_INVALID;
  }
  c->max_nc = o.max_nc_qubits ? o.max_nc_qubits : 12;
  c->max_cuts = o.max_cuts ? o.max_cuts : 12;
  if (c->max_nc > (uint32_t)kMaxNcQubits) {
    g_create_err = "max_nc_qubits above 12 (LDS state vector limit)";
    return CCUT_E_UNSUPPORTED;
  }
  if (c->device >= 0) {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || c->device >= n) {
      g_create_err = "no such HIP device";
      return CCUT_E_DEVICE;
    }
    if (hipSetDevice(c->device) != hipSuccess) {
      g_create_err = "hipSetDevice failed";
      return CCUT_E_DEVICE;
    }
  }
  *out = c.release();
  return CCUT_OK;
}

}  // extern "C"

namespace {
void ctx_free(ccut_ctx *c) {
  if (c->device >= 0) {
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (auto &pt : c->pending) {
      (void)hipEventDestroy(pt.a);
      (void)hipEventDestroy(pt.b);
    }
    for (auto e : c->event_pool) (void)hipEventDestroy(e);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->aux) {
      (void)hipStreamSynchronize(c->aux);
      (void)hipStreamDestroy(c->aux);
      (void)hipEventDestroy(c->fork_ev);
      (void)hipEventDestroy(c->join_ev);
    }
    c->arena.release();
    for (auto &sl : c->pin) {
      for (auto &ch : sl.chunks) (void)hipHostFree(ch.first);
      if (sl.ev_s) (void)hipEventDestroy(sl.ev_s);
      if (sl.ev_a) (void)hipEventDestroy(sl.ev_a);
    }
  }
  delete c;
}
}  // namespace

namespace {
// Objects created from a context keep it alive: its release waits for the
// last of them.
void ctx_retain(ccut_ctx *c) { ++c->children; }
void ctx_release(ccut_ctx *c) {
  if (c && --c->children == 0 && c->closed) ctx_free(c);
}
}  // namespace

extern "C" {

void ccut_ctx_destroy(ccut_ctx *c) {
  if (!c) return;
  if (c->children > 0) {
    c->closed = true;
    return;
  }
  ctx_free(c);
}

const char *ccut_last_error(const ccut_ctx *c) { return c ? c->err.c_str() : g_create_err.c_str(); }

void ccut_cancel(ccut_ctx *c) {
  if (c) c->cancel.store(1);
}

ccut_status ccut_plan_create(ccut_ctx *c, uint32_t n_qubits, const ccut_op *ops, size_t n_ops,
                             const ccut_cut *cuts, size_t k, ccut_plan **out) {
  if (!c || !out || (n_ops && !ops) || (k && !cuts)) return fail(c, CCUT_E_INVALID, "NULL argument");
  *out = nullptr;
  std::vector<HostOp> hops(n_ops);
  for (size_t i = 0; i < n_ops; ++i) hops[i] = {ops[i].kind, ops[i].q0, ops[i].q1, ops[i].theta};
  std::vector<uint32_t> cq(k), ca(k);
  for (size_t i = 0; i < k; ++i) {
    cq[i] = cuts[i].qubit;
    ca[i] = cuts[i].after_op;
  }
  std::unique_ptr<ccut_plan> p(new (std::nothrow) ccut_plan());
  if (!p) return fail(c, CCUT_E_OOM, "host allocation failed");
  p->ctx = c;
  std::string err;
  int st = build_plan(n_qubits, hops.data(), n_ops, cq.data(), ca.data(), k, c->max_nc, c->max_cuts, p->pd,
                      err);
  if (st != CCUT_OK) return fail(c, (ccut_status)st, err);
  *out = p.release();
  ctx_retain(c);
  c->err.clear();
  return CCUT_OK;
}

void ccut_plan_destroy(ccut_plan *p) {
  if (!p) return;
  ccut_ctx *c = p->ctx;
  if (c && c->device >= 0) (void)hipSetDevice(c->device);
  delete p;
  ctx_release(c);
}

ccut_status ccut_plan_info(const ccut_plan *p, uint32_t *nf, uint64_t *nv, uint64_t *nt) {
  if (!p) return CCUT_E_INVALID;
  uint64_t v = 0;
  for (const Fragment &f : p->pd.frags) v += f.n_variants;
  if (nf) *nf = (uint32_t)p->pd.frags.size();
  if (nv) *nv = v;
  if (nt) *nt = 1ull << (2 * p->pd.k);
  return CCUT_OK;
}

ccut_status ccut_fragment_info(const ccut_plan *p, uint32_t f, uint32_t *m, int32_t *cl, uint32_t *na,
                               uint64_t *nv) {
  if (!p || f >= p->pd.frags.size()) return CCUT_E_INVALID;
  const Fragment &F = p->pd.frags[f];
  if (m) *m = F.m();
  if (cl) *cl = F.clifford ? 1 : 0;
  if (na) *na = (uint32_t)F.axes.size();
  if (nv) *nv = F.n_variants;
  return CCUT_OK;
}

ccut_status ccut_fragment_segments(const ccut_plan *p, uint32_t f, uint32_t *wires, uint32_t *segs) {
  if (!p || f >= p->pd.frags.size()) return CCUT_E_INVALID;
  const Fragment &F = p->pd.frags[f];
  for (uint32_t i = 0; i < F.m(); ++i) {
    if (wires) wires[i] = F.wires[i];
    if (segs) segs[i] = F.segs[i];
  }
  return CCUT_OK;
}

ccut_status ccut_fragment_axes(const ccut_plan *p, uint32_t f, uint32_t *cut, uint32_t *side,
                               uint32_t *local) {
  if (!p || f >= p->pd.frags.size()) return CCUT_E_INVALID;
  const Fragment &F = p->pd.frags[f];
  for (size_t j = 0; j < F.axes.size(); ++j) {
    if (cut) cut[j] = F.axes[j].cut;
    if (side) side[j] = F.axes[j].side;
    if (local) local[j] = F.axes[j].local;
  }
  return CCUT_OK;
}

ccut_status ccut_fragment_ops(const ccut_plan *p, uint32_t f, uint32_t *n_one, uint32_t *n_two) {
  if (!p || f >= p->pd.frags.size()) return CCUT_E_INVALID;
  const Fragment &F = p->pd.frags[f];
  const std::vector<uint32_t> &w = F.clifford ? F.cl_words : F.sv_words;
  uint32_t one = 0, two = 0;
  for (uint32_t x : w) {
    const uint32_t k = op_kind(x);
    if (k == G_CX || k == G_CZ)
      ++two;
    else if (k != G_NOP)
      ++one;
  }
  if (n_one) *n_one = one;
  if (n_two) *n_two = two;
  return CCUT_OK;
}

ccut_status ccut_request_info(ccut_plan *p, const uint32_t *qubits, uint32_t nq, uint32_t fragment,
                              uint32_t *n_measured, uint32_t *n_requested) {
  if (!p || fragment >= p->pd.frags.size()) return CCUT_E_INVALID;
  ccut_status st = check_request(p->ctx, p->pd.n, qubits, nq, p->pd.n);
  if (st != CCUT_OK) return st;
  FragRequest r = marginal_request(p->pd.frags[fragment], qubits, nq);
  if (n_measured) *n_measured = (uint32_t)r.meas.size();
  if (n_requested) *n_requested = (uint32_t)r.req_pos.size();
  return CCUT_OK;
}

ccut_status ccut_variant_tables(ccut_plan *p, const ccut_eval_opts *eo, const uint32_t *qubits, uint32_t nq,
                                uint32_t fragment, double *out, int on_device) {
  ccut_status st = check_eval(p, eo);
  if (st != CCUT_OK) return st;
  ccut_ctx *c = p->ctx;
  if (eo->flags & CCUT_FLAG_SKIP) return fail(c, CCUT_E_UNSUPPORTED, "variant skipping applies to marginals");
  if (fragment >= p->pd.frags.size()) return fail(c, CCUT_E_INVALID, "fragment out of range");
  if ((st = check_request(c, p->pd.n, qubits, nq, p->pd.n)) != CCUT_OK) return st;
  const Fragment &f = p->pd.frags[fragment];
  FragRequest r = marginal_request(f, qubits, nq);
  double *dist = nullptr;
  if ((st = variant_dists(p, eo, f, r, &dist)) != CCUT_OK) return st;
  return finish_out(c, dist, out, (size_t)(f.n_variants << r.meas.size()), on_device);
}

ccut_status ccut_fragment_tensor(ccut_plan *p, const ccut_eval_opts *eo, const uint32_t *qubits, uint32_t nq,
                                 uint32_t fragment, double *out, int on_device) {
  ccut_status st = check_eval(p, eo);
  if (st != CCUT_OK) return st;
  ccut_ctx *c = p->ctx;
  if (eo->flags & CCUT_FLAG_SKIP) return fail(c, CCUT_E_UNSUPPORTED, "variant skipping applies to marginals");
  if (fragment >= p->pd.frags.size()) return fail(c, CCUT_E_INVALID, "fragment out of range");
  if ((st = check_request(c, p->pd.n, qubits, nq, p->pd.n)) != CCUT_OK) return st;
  const Fragment &f = p->pd.frags[fragment];
  FragRequest r = marginal_request(f, qubits, nq);
  double *dist = nullptr, *T = nullptr;
  if (use_heisenberg(f, eo, r.req_pos.size())) {
    if ((st = heis_tensor(p, f, r, eo->circuit, nullptr, &T)) != CCUT_OK) return st;
  } else {
    if ((st = variant_dists(p, eo, f, r, &dist)) != CCUT_OK) return st;
    if ((st = pauli_passes(c, f, r, dist, 1ull << r.meas.size(), 0, &T)) != CCUT_OK) return st;
  }
  size_t count = ((size_t)1 << (2 * f.axes.size())) << r.req_pos.size();
  return finish_out(c, T, out, count, on_device);
}

}  // extern "C"

namespace {
// Enqueue the whole marginal evaluation of one plan (no final copy, no
// sync); res receives 2^nq doubles.  pre_models[f], if given, holds the
// already computed sample models of Clifford fragment f.
// The fragment whose variant tables stand in for its Pauli-basis tensor:
// the fragment with the most requested outputs (the contraction's column
// side, the largest tensor) when every cut axis of it is a quantum input
// and its tensor would come from variant tables.  Its preparation
// coefficients then move across the sum over each cut's Pauli onto the
// upstream fragment (fold_jobs), and its own transform is skipped (the
// sparse contraction then reads its support over these folded terms: a
// skipped term is still an exact zero).  -1: none.
int fold_target(const PlanData &pd, const ccut_eval_opts *eo, const uint32_t *qubits, uint32_t nq) {
  if (eo->flags & CCUT_FLAG_SKIP) return -1;  // every tensor in the Pauli basis: the support indexes Paulis
  int best = -1;
  size_t best_bits = 0;
  for (const Fragment &f : pd.frags) {
    const size_t bits = marginal_request(f, qubits, nq).req_pos.size();
    if (best < 0 || bits > best_bits) {
      best = (int)f.index;
      best_bits = bits;
    }
  }
  if (best < 0) return -1;
  const Fragment &g = pd.frags[best];
  if (g.axes.empty() || use_heisenberg(g, eo, best_bits)) return -1;
  for (const Axis &a : g.axes)
    if (a.side != 1) return -1;
  return best;
}

// Whether the fold target's tensor may stay 16-bit shot counts: sampled
// (fewer than 2^16 shots), read by the matrix contraction paths (not the
// plain sum, not the sparse support search).
bool counts_contraction(const PlanData &pd, const ccut_eval_opts *eo, uint32_t nq) {
  if (eo->shots_per_variant == 0 || eo->shots_per_variant > 0xFFFFull || (eo->flags & (CCUT_FLAG_SPARSE | CCUT_FLAG_SKIP)))
    return false;
  const uint64_t K = 1ull << (2 * pd.k);
  const bool fp32 = eo->precision != CCUT_FP64;
  return !(!fp32 && pd.frags.size() > 2 && (K << nq) <= (1ull << 20));
}

// The axes of fragment f on a cut of fragment g (bit j: axis j).
uint32_t fold_mask(const PlanData &pd, int g, const Fragment &f) {
  if (g < 0 || (int)f.index == g) return 0;
  uint32_t mask = 0;
  for (size_t j = 0; j < f.axes.size(); ++j)
    for (const Axis &a : pd.frags[g].axes)
      if (a.cut == f.axes[j].cut) mask |= 1u << j;
  return mask;
}

// The fold jobs of the other fragments: every axis on a cut of fragment g.
// folded[f] set: fragment f's tensor was folded where it was produced.
void fold_jobs(const PlanData &pd, int g, const RecombArgs &args, std::vector<FoldJob> &jobs,
               const std::vector<char> *folded = nullptr) {
  if (g < 0) return;
  for (const Fragment &f : pd.frags) {
    if (folded && (*folded)[f.index]) continue;
    const uint32_t mask = fold_mask(pd, g, f);
    const RecombFrag &rf = args.f[f.index];
    if (mask) jobs.push_back({const_cast<double *>(rf.T), rf.rows, rf.n_axes, mask});
  }
}

// Sec. IX, fewer downstream evaluations (CCUT_FLAG_SKIP): the support is
// fixed first from the Clifford fragments' exact Pauli tensors (Heisenberg
// picture where it applies, else exact variant tables); every sampled
// Clifford variant no term of the support reads draws no shots; the
// tensors are formed in the Pauli basis (no fold) and only the support's
// terms are summed.  The support size is read back (the call synchronizes).
ccut_status marginal_skip_enqueue(ccut_plan *p, const ccut_eval_opts *eo, const uint32_t *qubits, uint32_t nq,
                                  double *res) {
  ccut_ctx *c = p->ctx;
  ccut_status st;
  const PlanData &pd = p->pd;
  if (pd.frags.size() > (size_t)kMaxFrags) return fail(c, CCUT_E_UNSUPPORTED, "more than 64 fragments");
  const uint64_t K = 1ull << (2 * pd.k);
  const bool fp32 = eo->precision != CCUT_FP64;
  ccut_eval_opts ex = *eo;  // exact data for the support
  ex.shots_per_variant = 0;
  ex.flags = 0;
  ex.method = CCUT_METHOD_AUTO;
  RecombArgs sargs{};
  sargs.n_frags = (uint32_t)pd.frags.size();
  sargs.k = pd.k;
  SupportArgs sa{};
  uint64_t cols_total = 0;
  for (const Fragment &f : pd.frags) {
    sa.off[f.index] = cols_total;
    cols_total += 1ull << (2 * f.axes.size());
    sargs.f[f.index].n_axes = (uint32_t)f.axes.size();
    for (size_t j = 0; j < f.axes.size(); ++j) sargs.f[f.index].axis_cut[j] = f.axes[j].cut;
  }
  uint8_t *nz = aget<uint8_t>(c, cols_total);
  uint64_t *pos = aget<uint64_t>(c, K), *scratch = aget<uint64_t>(c, scan_scratch_words(K));
  uint64_t *terms = aget<uint64_t>(c, K);
  if (!nz || !pos || !scratch || !terms) return fail(c, CCUT_E_OOM, "device allocation failed");
  // each Clifford fragment's exact tensor, reused below for exact data
  // formed the same way
  std::vector<double *> ex_T(pd.frags.size(), nullptr);
  std::vector<uint8_t> ex_heis(pd.frags.size(), 0);
  for (const Fragment &f : pd.frags) {
    const uint64_t cols = 1ull << (2 * f.axes.size());
    if (!f.clifford) {  // a non-Clifford fragment does not restrict the support
      HIP_TRY(c, hipMemsetAsync(nz + sa.off[f.index], 1, cols, c->cur));
      continue;
    }
    FragRequest r = marginal_request(f, qubits, nq);
    double *T = nullptr;
    ex_heis[f.index] = use_heisenberg(f, &ex, r.req_pos.size());
    if (ex_heis[f.index]) {
      if ((st = heis_tensor(p, f, r, eo->circuit, nullptr, &T)) != CCUT_OK) return st;
    } else {
      double *dist0 = nullptr;
      if ((st = variant_dists(p, &ex, f, r, &dist0)) != CCUT_OK) return st;
      if ((st = pauli_passes(c, f, r, dist0, 1ull << r.meas.size(), 0, &T)) != CCUT_OK) return st;
    }
    ex_T[f.index] = T;
    KTimer t(c, CCUT_K_RECOMBINE);
    HIP_TRY(c, launch_colnz(T, 1u << r.req_pos.size(), cols, nz + sa.off[f.index], c->cur));
  }
  RecombArgs *dsargs = (RecombArgs *)upload(c, &sargs, sizeof(sargs));
  if (!dsargs) return fail(c, CCUT_E_OOM, "device allocation failed");
  {
    KTimer t(c, CCUT_K_RECOMBINE);
    HIP_TRY(c, launch_support_terms(dsargs, sa, nz, K, pos, scratch, terms, c->cur));
  }
  uint64_t count = 0;
  HIP_TRY(c, hipMemcpyAsync(&count, pos + K - 1, 8, hipMemcpyDeviceToHost, c->cur));
  HIP_TRY(c, hipStreamSynchronize(c->cur));
  std::vector<uint64_t> S(count);
  if (count) {
    HIP_TRY(c, hipMemcpyAsync(S.data(), terms, count * 8, hipMemcpyDeviceToHost, c->cur));
    HIP_TRY(c, hipStreamSynchronize(c->cur));
  }
  // the tensors, sampled Clifford variants restricted to the ones the
  // support reads: per axis, a quantum input's |0> and |1> serve every
  // Pauli, |+> X and |+i> Y; a quantum output's Z basis serves I and Z, X X
  // and Y Y
  RecombArgs args{};
  args.n_frags = (uint32_t)pd.frags.size();
  args.k = pd.k;
  args.lo_parts = eo->precision == CCUT_FP32X3_MFMA_FP64SUM;
  for (const Fragment &f : pd.frags) {
    route(c, f);
    FragRequest r = marginal_request(f, qubits, nq);
    double *T = nullptr;
    const bool heis = use_heisenberg(f, eo, r.req_pos.size());
    if (f.clifford && eo->shots_per_variant == 0 && heis == (bool)ex_heis[f.index]) {
      T = ex_T[f.index];
    } else if (heis) {
      if ((st = heis_tensor(p, f, r, eo->circuit, nullptr, &T)) != CCUT_OK) return st;
    } else {
      const uint8_t *vmask = nullptr;
      if (f.clifford && eo->shots_per_variant > 0) {
        // R[key] over the fragment's Pauli keys (2 bits per axis): some
        // support term projects to key.  Per axis, the four Pauli values are
        // then replaced by the three variant classes that read them: a
        // quantum input's {|0>,|1>} read every Pauli, |+> X and |+i> Y; a
        // quantum output's X basis X, Y basis Y and Z basis I and Z.  After
        // all axes R[c] says whether a variant of classes c is read.
        const size_t a = f.axes.size();
        std::vector<uint8_t> R(size_t(1) << (2 * a), 0);
        for (uint64_t P : S) {
          uint64_t key = 0;
          for (size_t j = 0; j < a; ++j) key |= ((P >> (2 * f.axes[j].cut)) & 3ull) << (2 * j);
          R[key] = 1;
        }
        for (size_t j = 0; j < a; ++j) {
          const size_t stride = size_t(1) << (2 * j);
          const bool in = f.axes[j].side == 1;
          for (size_t hi = 0; hi < R.size(); hi += 4 * stride)  // every index whose digit j is 0
            for (size_t base = hi; base < hi + stride; ++base) {
              const uint8_t pi = R[base], px = R[base + stride], py = R[base + 2 * stride], pz = R[base + 3 * stride];
              if (in) {
                R[base] = pi | px | py | pz;  // |0>, |1>
                R[base + stride] = px;        // |+>
                R[base + 2 * stride] = py;    // |+i>
              } else {
                R[base] = px;                 // X basis
                R[base + stride] = py;        // Y basis
                R[base + 2 * stride] = pi | pz;  // Z basis
              }
              R[base + 3 * stride] = 0;
            }
        }
        // variant v's digits counted up in mixed radix (axis 0 fastest), its
        // class index kept alongside
        static const uint32_t kPrepClass[4] = {0, 0, 1, 2};  // |0> |1> |+> |+i>
        std::vector<uint8_t> need(f.n_variants, 0);
        std::vector<uint32_t> dig(a, 0);
        uint64_t cls = 0;
        for (uint64_t v = 0; v < f.n_variants; ++v) {
          need[v] = R[cls];
          for (size_t j = 0; j < a; ++j) {
            const bool in = f.axes[j].side == 1;
            const uint32_t rad = in ? 4u : 3u;
            dig[j] = dig[j] + 1 == rad ? 0u : dig[j] + 1;
            const uint32_t c_j = in ? kPrepClass[dig[j]] : dig[j];  // bases X=0 Y=1 Z=2
            cls = (cls & ~(3ull << (2 * j))) | ((uint64_t)c_j << (2 * j));
            if (dig[j] != 0) break;  // no carry into the next axis
          }
        }
        vmask = (const uint8_t *)upload(c, need.data(), need.size());
        if (!vmask) return fail(c, CCUT_E_OOM, "device allocation failed");
      }
      double *dist = nullptr;
      if ((st = variant_dists(p, eo, f, r, &dist, nullptr, nullptr, vmask)) != CCUT_OK) return st;
      if (f.axes.empty())
        T = dist;
      else if ((st = pauli_passes(c, f, r, dist, 1ull << r.meas.size(), 0, &T)) != CCUT_OK)
        return st;
    }
    RecombFrag &rf = args.f[f.index];
    rf.T = T;
    rf.n_axes = (uint32_t)f.axes.size();
    rf.rows = 1u << r.req_pos.size();
    rf.n_req = (uint32_t)r.req_pos.size();
    for (size_t j = 0; j < f.axes.size(); ++j) rf.axis_cut[j] = f.axes[j].cut;
    for (size_t i = 0; i < r.req_user.size(); ++i) rf.req_user[i] = r.req_user[i];
    if ((st = cancelled(c)) != CCUT_OK) return st;
  }
  if ((st = join(c)) != CCUT_OK) return st;
  RecombArgs *dargs = (RecombArgs *)upload(c, &args, sizeof(args));
  if (!dargs) return fail(c, CCUT_E_OOM, "device allocation failed");
  return contract_terms(c, args, dargs, nq, fp32, res, terms, count);
}

ccut_status marginal_enqueue(ccut_plan *p, const ccut_eval_opts *eo, const uint32_t *qubits, uint32_t nq,
                             double *res, const std::vector<uint64_t *> *pre_models,
                             const std::vector<double *> *pre_dist = nullptr) {
  ccut_ctx *c = p->ctx;
  ccut_status st;
  const PlanData &pd = p->pd;
  if (pd.frags.size() > (size_t)kMaxFrags) return fail(c, CCUT_E_UNSUPPORTED, "more than 64 fragments");
  RecombArgs args{};
  args.n_frags = (uint32_t)pd.frags.size();
  args.k = pd.k;
  args.lo_parts = eo->precision == CCUT_FP32X3_MFMA_FP64SUM;
  const int g = fold_target(pd, eo, qubits, nq);
  const bool counts_ok = counts_contraction(pd, eo, nq);
  for (const Fragment &f : pd.frags) {
    route(c, f);
    FragRequest r = marginal_request(f, qubits, nq);
    double *dist = nullptr, *T = nullptr;
    if (use_heisenberg(f, eo, r.req_pos.size())) {
      if ((st = heis_tensor(p, f, r, eo->circuit, nullptr, &T)) != CCUT_OK) return st;
    } else {
      uint64_t *pm = pre_models ? (*pre_models)[f.index] : nullptr;
      dist = pre_dist ? (*pre_dist)[f.index] : nullptr;
      uint16_t *cnt = nullptr;
      const bool counts = (int)f.index == g && counts_ok;
      if (!dist && (st = variant_dists(p, eo, f, r, &dist, pm, counts ? &cnt : nullptr)) != CCUT_OK) return st;
      if ((int)f.index == g)
        T = cnt ? reinterpret_cast<double *>(cnt) : dist;  // tables [preparations][outcomes]: the tensor's layout
      else if ((st = pauli_passes(c, f, r, dist, 1ull << r.meas.size(), 0, &T)) != CCUT_OK)
        return st;
      if (cnt) {
        args.f[f.index].cnt16 = 1;
        args.f[f.index].shots = (double)eo->shots_per_variant;
      }
    }
    RecombFrag &rf = args.f[f.index];
    rf.T = T;
    rf.n_axes = (uint32_t)f.axes.size();
    rf.rows = 1u << r.req_pos.size();
    rf.n_req = (uint32_t)r.req_pos.size();
    for (size_t j = 0; j < f.axes.size(); ++j) rf.axis_cut[j] = f.axes[j].cut;
    for (size_t i = 0; i < r.req_user.size(); ++i) rf.req_user[i] = r.req_user[i];
    if ((st = cancelled(c)) != CCUT_OK) return st;
  }
  if ((st = join(c)) != CCUT_OK) return st;
  std::vector<FoldJob> fj;
  fold_jobs(pd, g, args, fj);
  if (!fj.empty()) {
    FoldJob *d_fj = (FoldJob *)upload(c, fj.data(), fj.size() * sizeof(FoldJob));
    if (!d_fj) return fail(c, CCUT_E_OOM, "device allocation failed");
    KTimer t(c, CCUT_K_TRANSFORM);
    HIP_TRY(c, launch_fold(d_fj, (uint32_t)fj.size(), c->cur));
  }
  return recombine(c, args, nq, eo->precision != CCUT_FP64, res, (eo->flags & CCUT_FLAG_SPARSE) != 0);
}
}  // namespace

namespace {

void key_put(std::vector<uint8_t> &k, const void *src, size_t n) {
  k.insert(k.end(), (const uint8_t *)src, (const uint8_t *)src + n);
}

// Argument key of a call: entry point, every option, the request and the
// output address.
std::vector<uint8_t> call_key(uint32_t entry, const ccut_eval_opts *eo, const void *req, size_t req_bytes,
                              const double *out) {
  std::vector<uint8_t> k;
  key_put(k, &entry, 4);
  key_put(k, &eo->seed, 8);
  key_put(k, &eo->shots_per_variant, 8);
  key_put(k, &eo->precision, 4);
  key_put(k, &eo->circuit, 4);
  key_put(k, &eo->method, 4);
  key_put(k, &eo->flags, 4);
  key_put(k, &req_bytes, sizeof(req_bytes));
  key_put(k, req, req_bytes);
  const uintptr_t o = (uintptr_t)out;
  key_put(k, &o, sizeof(o));
  return k;
}

// Run a device-output call through the plan's call graphs: the first call
// with a given key runs eagerly, the second is captured (every launch and
// copy it enqueues, on both streams) and replayed, later ones only replay.
// Calls with host outputs, with kernel timing on, or issued while the
// caller's stream is itself being captured always run eagerly.  The graph's
// scratch lives in the context's pool, which only grows, so its addresses
// stay valid; replays and eager calls are ordered on the context's stream.
template <class Impl>
ccut_status graph_call(ccut_plan *p, std::vector<uint8_t> &&key, int on_device, Impl &&impl) {
  ccut_ctx *c = p ? p->ctx : nullptr;
  if (!c || !on_device || !c->call_graphs || c->timing || c->device < 0 || c->capturing) return impl();
  if (hipSetDevice(c->device) != hipSuccess) return impl();
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(c->stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return impl();
  CallGraph *g = nullptr;
  for (auto &e : p->graphs)
    if (e.key == key) g = &e;
  if (g && g->no_graph) return impl();
  if (g && g->exec) {
    g->last_use = ++p->graph_tick;
    c->cancel.store(0);
    HIP_TRY(c, hipGraphLaunch(g->exec, c->stream));
    return CCUT_OK;
  }
  if (!g) {  // first sighting: eager, remembered only if it succeeds
    ccut_status st = impl();
    if (st != CCUT_OK) return st;
    if (p->graphs.size() >= ccut_plan::kMaxCallGraphs) {
      auto lru = std::min_element(p->graphs.begin(), p->graphs.end(),
                                  [](const CallGraph &a, const CallGraph &b) { return a.last_use < b.last_use; });
      (void)hipStreamSynchronize(c->stream);  // a replay of it may still be running
      lru->release();
      p->graphs.erase(lru);
    }
    p->graphs.emplace_back();
    CallGraph &e = p->graphs.back();
    e.key = std::move(key);
    e.upload_bytes = c->call_upload_bytes;
    e.last_use = ++p->graph_tick;
    return CCUT_OK;
  }
  // second sighting: capture, instantiate, launch
  g->last_use = ++p->graph_tick;
  g->pin_cap = std::max<size_t>(g->upload_bytes, 256);
  g->pin_used = 0;
  HIP_TRY(c, hipHostMalloc((void **)&g->pin, g->pin_cap, hipHostMallocDefault));
  HIP_TRY(c, hipMalloc((void **)&g->dev, g->pin_cap));
  // captured on a private stream (the caller's may be the legacy default
  // stream, which cannot be captured) and launched on the caller's
  if (!c->cap_stream) HIP_TRY(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  HIP_TRY(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
  const hipStream_t caller = c->stream;
  c->stream = c->cap_stream;
  c->capturing = g;
  c->arena.frozen = true;
  ccut_status st = impl();
  c->arena.frozen = false;
  c->capturing = nullptr;
  c->stream = caller;
  hipGraph_t graph = nullptr;
  const hipError_t e_end = hipStreamEndCapture(c->cap_stream, &graph);
  hipError_t e_inst = hipErrorUnknown;
  if (st == CCUT_OK && e_end == hipSuccess && graph) e_inst = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
  if (graph) (void)hipGraphDestroy(graph);
  if (st != CCUT_OK || e_inst != hipSuccess) {
    // stay eager for this key; the capture enqueued nothing, so run the call now
    g->release();
    g->no_graph = true;
    (void)hipGetLastError();
    return impl();
  }
  if (g->pin_used) HIP_TRY(c, hipMemcpyAsync(g->dev, g->pin, g->pin_used, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipGraphLaunch(g->exec, c->stream));
  return CCUT_OK;
}

ccut_status marginal_call(ccut_plan *p, const ccut_eval_opts *eo, const uint32_t *qubits, uint32_t nq,
                          double *out, int on_device) {
  ccut_status st = check_eval(p, eo);
  if (st != CCUT_OK) return st;
  ccut_ctx *c = p->ctx;
  if (!out) return fail(c, CCUT_E_INVALID, "out is NULL");
  if (eo->flags & CCUT_FLAG_SETTLE) return fail(c, CCUT_E_UNSUPPORTED, "settlement applies to Z-string expectations");
  if ((st = check_request(c, p->pd.n, qubits, nq)) != CCUT_OK) return st;
  // a device output receives the contraction directly
  double *res = on_device ? out : aget<double>(c, (size_t)1 << nq);
  if (!res) return fail(c, CCUT_E_OOM, "device allocation failed");
  if (eo->flags & CCUT_FLAG_SKIP) {
    if (eo->flags & CCUT_FLAG_ML)
      return fail(c, CCUT_E_UNSUPPORTED, "the maximum-likelihood correction needs every variant (no skipping)");
    st = marginal_skip_enqueue(p, eo, qubits, nq, res);
  } else {
    st = marginal_enqueue(p, eo, qubits, nq, res, nullptr);
  }
  if (st != CCUT_OK) return st;
  return on_device ? CCUT_OK : finish_out(c, res, out, (size_t)1 << nq, on_device);
}

ccut_status zexpect_call(ccut_plan *p, const ccut_eval_opts *eo, const uint64_t *masks, uint32_t n_strings,
                         double *out, int on_device) {
  ccut_status st = check_eval(p, eo);
  if (st != CCUT_OK) return st;
  ccut_ctx *c = p->ctx;
  if (!out || (n_strings && !masks)) return fail(c, CCUT_E_INVALID, "NULL argument");
  if (eo->flags & (CCUT_FLAG_SPARSE | CCUT_FLAG_SKIP))
    return fail(c, CCUT_E_UNSUPPORTED, "the sparse contraction and variant skipping apply to marginals");
  if (eo->flags & CCUT_FLAG_ML) return fail(c, CCUT_E_UNSUPPORTED, "the maximum-likelihood correction applies to outcome tables");
  if (n_strings == 0) return CCUT_OK;
  const PlanData &pd = p->pd;
  if (pd.frags.size() > (size_t)kMaxFrags) return fail(c, CCUT_E_UNSUPPORTED, "more than 64 fragments");
  const uint32_t nw = (pd.n + 63) / 64;
  std::vector<uint64_t> anymask(nw, 0);
  for (uint32_t s = 0; s < n_strings; ++s)
    for (uint32_t w = 0; w < nw; ++w) anymask[w] |= masks[(size_t)s * nw + w];
  if (nw && (pd.n & 63) && (anymask[nw - 1] >> (pd.n & 63)))
    return fail(c, CCUT_E_INVALID, "mask bit beyond n_qubits");
  RecombArgs args{};
  args.n_frags = (uint32_t)pd.frags.size();
  args.k = pd.k;
  args.lo_parts = eo->precision == CCUT_FP32X3_MFMA_FP64SUM;
  for (const Fragment &f : pd.frags) {
    route(c, f);
    FragRequest r = zstring_request(f, anymask);
    const uint32_t nm = (uint32_t)r.meas.size();
    const uint64_t nv = f.n_variants;
    if (use_heisenberg(f, eo, 0)) {
      const uint32_t W = row_words(f.m());
      if (!W) return fail(c, CCUT_E_UNSUPPORTED, "Clifford fragment wider than 512 qubits");
      std::vector<std::vector<uint64_t>> zs(n_strings, std::vector<uint64_t>(W, 0));
      for (uint32_t s2 = 0; s2 < n_strings; ++s2)
        for (uint32_t q = 0; q < pd.n; ++q) {
          const int32_t l = f.out_local[q];
          if (l >= 0 && ((masks[(size_t)s2 * nw + (q >> 6)] >> (q & 63)) & 1ull))
            zs[s2][l >> 6] |= 1ull << (l & 63);
        }
      double *T = nullptr;
      if ((st = heis_tensor(p, f, r, eo->circuit, &zs, &T)) != CCUT_OK) return st;
      RecombFrag &rf = args.f[f.index];
      rf.T = T;
      rf.n_axes = (uint32_t)f.axes.size();
      rf.rows = n_strings;
      rf.n_req = 0;
      for (size_t j = 0; j < f.axes.size(); ++j) rf.axis_cut[j] = f.axes[j].cut;
      continue;
    }
    // a non-Clifford fragment's tables, or a Clifford fragment's models
    // (one outcome vector of MW words; more than 64 measurements: wide)
    if (!f.clifford && nm > (uint32_t)kMaxTableBits)
      return fail(c, CCUT_E_UNSUPPORTED, "outcome table over more than 24 measured qubits");
    if (nm > (uint32_t)kMaxMeasWide) return fail(c, CCUT_E_UNSUPPORTED, "more than 1024 measured qubits in a fragment");
    const bool wide = nm > (uint32_t)kMaxMeas;
    const uint32_t MW = model_mw(nm);
    // extended masks [J][string][MW words] over measured positions
    std::vector<uint32_t> outpos;
    for (size_t j = 0; j < f.axes.size(); ++j)
      if (f.axes[j].side == 0) outpos.push_back((uint32_t)r.axis_outpos[j]);
    const uint32_t n_out = (uint32_t)outpos.size();
    if (n_out > 12) return fail(c, CCUT_E_UNSUPPORTED, "more than 12 quantum outputs in a fragment");
    const uint32_t n_ext = n_strings << n_out;
    std::vector<uint64_t> ext((size_t)n_ext * MW, 0);
    for (uint32_t s = 0; s < n_strings; ++s) {
      std::vector<uint64_t> z(MW, 0);
      for (uint32_t jpos = 0; jpos < nm; ++jpos) {
        const uint32_t wire = f.wires[r.meas[jpos]];
        const bool is_cout = f.out_local[wire] == (int32_t)r.meas[jpos];
        if (is_cout && ((masks[(size_t)s * nw + (wire >> 6)] >> (wire & 63)) & 1ull)) z[jpos >> 6] |= 1ull << (jpos & 63);
      }
      for (uint32_t J = 0; J < (1u << n_out); ++J) {
        uint64_t *e = &ext[((size_t)J * n_strings + s) * MW];
        for (uint32_t w = 0; w < MW; ++w) e[w] = z[w];
        for (uint32_t i = 0; i < n_out; ++i)
          if ((J >> i) & 1u) e[outpos[i] >> 6] |= 1ull << (outpos[i] & 63);
      }
    }
    uint64_t *d_ext = (uint64_t *)upload(c, ext.data(), ext.size() * 8);
    double *E = aget<double>(c, nv * n_ext);
    if (!d_ext || !E) return fail(c, CCUT_E_OOM, "device allocation failed");
    const FragDev h = frag_desc(p, f, r, eo->circuit);
    if (!f.clifford) {
      double *dist = aget<double>(c, nv << nm);
      const size_t sb = sv_states_bytes(h);
      double *states = sb ? aget<double>(c, sb / sizeof(double)) : nullptr;
      if (!dist || (sb && !states)) return fail(c, CCUT_E_OOM, "device allocation failed");
      {
        KTimer t(c, CCUT_K_SV);
        HIP_TRY(c, launch_sv(h, dist, states, c->cur));
      }
      KTimer t(c, CCUT_K_PARITY);
      HIP_TRY(c, launch_dist_parity(dist, nm, nv, d_ext, n_ext, E, c->cur));
    } else {
      uint64_t *models = aget<uint64_t>(c, nv * model_words(nm));
      if (!models) return fail(c, CCUT_E_OOM, "device allocation failed");
      {
        ccut_status st2 = tableau_models(p, f, h, r, 0, nv, models);
        if (st2 != CCUT_OK) return st2;
      }
      if (eo->shots_per_variant == 0) {
        KTimer t(c, CCUT_K_PARITY);
        if (wide)
          HIP_TRY(c, launch_parity_exact_wide(models, nm, nv, d_ext, n_ext, E, c->cur));
        else
          HIP_TRY(c, launch_parity_exact(models, nm, nv, d_ext, n_ext, E, c->cur));
      } else {
        uint32_t *odd = aget<uint32_t>(c, nv * n_ext);
        if (!odd) return fail(c, CCUT_E_OOM, "device allocation failed");
        HIP_TRY(c, launch_fill_u32(odd, nv * n_ext, 0u, c->cur));
        for (uint64_t v0 = 0; v0 < nv; v0 += 65535) {
          const uint64_t cnv = std::min<uint64_t>(65535, nv - v0);
          KTimer t(c, CCUT_K_PARITY);
          if (wide)
            HIP_TRY(c, launch_parity_sampled_wide(models + v0 * model_words(nm), nm, cnv, eo->shots_per_variant,
                                                  eo->seed, h.vid_base + v0, d_ext, n_ext, odd + v0 * n_ext,
                                                  c->cur));
          else
            HIP_TRY(c, launch_parity_sampled(models + v0 * model_words(nm), nm, cnv, eo->shots_per_variant,
                                             eo->seed, h.vid_base + v0, d_ext, n_ext, odd + v0 * n_ext,
                                             c->cur));
        }
        HIP_TRY(c, launch_parity_finish(odd, nv * n_ext, eo->shots_per_variant, (eo->flags & CCUT_FLAG_SETTLE) != 0,
                                        E, c->cur));
      }
    }
    double *T = nullptr;
    if ((st = pauli_passes(c, f, r, E, n_ext, n_strings, &T)) != CCUT_OK) return st;
    RecombFrag &rf = args.f[f.index];
    rf.T = T;
    rf.n_axes = (uint32_t)f.axes.size();
    rf.rows = n_strings;
    rf.n_req = 0;
    for (size_t j = 0; j < f.axes.size(); ++j) rf.axis_cut[j] = f.axes[j].cut;
    if ((st = cancelled(c)) != CCUT_OK) return st;
  }
  if ((st = join(c)) != CCUT_OK) return st;
  RecombArgs *dargs = (RecombArgs *)upload(c, &args, sizeof(args));
  double *res = on_device ? out : aget<double>(c, n_strings);  // a device output receives the sums directly
  const uint32_t zsplits = zrecombine_splits(pd.k, n_strings);
  double *zpart = aget<double>(c, (size_t)zsplits * n_strings);
  if (!dargs || !res || !zpart) return fail(c, CCUT_E_OOM, "device allocation failed");
  {
    KTimer t(c, CCUT_K_ZRECOMBINE);
    HIP_TRY(c, launch_zrecombine(dargs, args.n_frags, pd.k, n_strings, eo->precision != CCUT_FP64,
                                 zpart, zsplits, res, c->cur));
  }
  return on_device ? CCUT_OK : finish_out(c, res, out, n_strings, on_device);
}

}  // namespace

extern "C" {

ccut_status ccut_marginal(ccut_plan *p, const ccut_eval_opts *eo, const uint32_t *qubits, uint32_t nq,
                          double *out, int on_device) {
  // a sparse or skipping contraction reads its support back: never captured
  if (!p || !eo || !out || (nq && !qubits) || nq > 24 || (eo->flags & (CCUT_FLAG_SPARSE | CCUT_FLAG_SKIP)))
    return marginal_call(p, eo, qubits, nq, out, on_device);
  return graph_call(p, call_key(0, eo, qubits, (size_t)nq * 4, out), on_device,
                    [&] { return marginal_call(p, eo, qubits, nq, out, on_device); });
}

ccut_status ccut_zexpect(ccut_plan *p, const ccut_eval_opts *eo, const uint64_t *masks, uint32_t n_strings,
                         double *out, int on_device) {
  if (!p || !eo || !out || !masks || n_strings == 0)
    return zexpect_call(p, eo, masks, n_strings, out, on_device);
  const size_t nw = (p->pd.n + 63) / 64;
  return graph_call(p, call_key(1, eo, masks, (size_t)n_strings * nw * 8, out), on_device,
                    [&] { return zexpect_call(p, eo, masks, n_strings, out, on_device); });
}

ccut_status ccut_call_graphs(ccut_ctx *c, int enable) {
  if (!c) return CCUT_E_INVALID;
  c->call_graphs = enable != 0;
  return CCUT_OK;
}

ccut_status ccut_shot_records(ccut_plan *p, const ccut_eval_opts *eo, const uint32_t *qubits, uint32_t nq,
                              uint32_t fragment, uint64_t v_begin, uint64_t v_end, uint64_t *out,
                              int on_device) {
  ccut_status st = check_eval(p, eo);
  if (st != CCUT_OK) return st;
  ccut_ctx *c = p->ctx;
  if (fragment >= p->pd.frags.size()) return fail(c, CCUT_E_INVALID, "fragment out of range");
  if ((st = check_request(c, p->pd.n, qubits, nq, p->pd.n)) != CCUT_OK) return st;
  const Fragment &f = p->pd.frags[fragment];
  if (!f.clifford) return fail(c, CCUT_E_INVALID, "shot records exist only for Clifford fragments");
  if (eo->flags) return fail(c, CCUT_E_UNSUPPORTED, "evaluation flags do not apply to shot records");
  if (eo->shots_per_variant == 0) return fail(c, CCUT_E_INVALID, "shot records need shots > 0");
  if (v_begin > v_end || v_end > f.n_variants) return fail(c, CCUT_E_INVALID, "bad variant range");
  const uint64_t nv = v_end - v_begin;
  if (nv == 0) return CCUT_OK;
  FragRequest r = marginal_request(f, qubits, nq);
  const uint32_t nm = (uint32_t)r.meas.size();
  if (nm > (uint32_t)kMaxMeasWide) return fail(c, CCUT_E_UNSUPPORTED, "more than 1024 measured qubits");
  const bool wide = nm > (uint32_t)kMaxMeas;
  const uint32_t RW = wide ? (nm + 63) / 64 : 1;  // record words
  const FragDev h = frag_desc(p, f, r, eo->circuit);
  uint64_t *models = aget<uint64_t>(c, nv * model_words(nm));
  const uint64_t shots = eo->shots_per_variant;
  uint64_t *rec = aget<uint64_t>(c, nv * shots * RW);
  if (!models || !rec) return fail(c, CCUT_E_OOM, "device allocation failed");
  if ((st = tableau_models(p, f, h, r, v_begin, nv, models)) != CCUT_OK) return st;
  const uint64_t nquads = (shots + 3) / 4;
  for (uint64_t v0 = 0; v0 < nv; v0 += 65535) {
    const uint64_t cnv = std::min<uint64_t>(65535, nv - v0);
    const uint32_t nblk = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((nquads + kSampleThreads - 1) / kSampleThreads, 4096));
    const uint32_t qpt = (uint32_t)((nquads + (uint64_t)nblk * kSampleThreads - 1) / ((uint64_t)nblk * kSampleThreads));
    KTimer t(c, CCUT_K_SAMPLE);
    if (wide)
      HIP_TRY(c, launch_records_wide(models + v0 * model_words(nm), nm, cnv, shots, eo->seed, h.vid_base + v_begin + v0,
                                     rec + v0 * shots * RW, c->cur));
    else
      HIP_TRY(c, launch_sample_hist(models + v0 * model_words(nm), nm, cnv, shots, eo->seed,
                                    h.vid_base + v_begin + v0, nullptr, nblk, qpt, rec + v0 * shots, c->cur));
  }
  HIP_TRY(c, hipMemcpyAsync(out, rec, nv * shots * RW * 8,
                            on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->cur));
  HIP_TRY(c, hipStreamSynchronize(c->cur));
  return CCUT_OK;
}

ccut_status ccut_timing_enable(ccut_ctx *c, int enable) {
  if (!c) return CCUT_E_INVALID;
  c->timing = enable != 0;
  return CCUT_OK;
}

static ccut_status drain_timing(ccut_ctx *c) {
  for (auto &pt : c->pending) {
    HIP_TRY(c, hipEventSynchronize(pt.b));
    float ms = 0.f;
    HIP_TRY(c, hipEventElapsedTime(&ms, pt.a, pt.b));
    c->launches[pt.kid] += 1;
    c->total_ms[pt.kid] += ms;
    c->event_pool.push_back(pt.a);
    c->event_pool.push_back(pt.b);
  }
  c->pending.clear();
  return CCUT_OK;
}

ccut_status ccut_timing_reset(ccut_ctx *c) {
  if (!c) return CCUT_E_INVALID;
  ccut_status st = drain_timing(c);
  for (int i = 0; i < CCUT_K_COUNT; ++i) {
    c->launches[i] = 0;
    c->total_ms[i] = 0;
  }
  return st;
}

ccut_status ccut_timing_read(ccut_ctx *c, uint32_t kid, uint64_t *launches, double *total_ms) {
  if (!c || kid >= CCUT_K_COUNT) return CCUT_E_INVALID;
  ccut_status st = drain_timing(c);
  if (st != CCUT_OK) return st;
  if (launches) *launches = c->launches[kid];
  if (total_ms) *total_ms = c->total_ms[kid];
  return CCUT_OK;
}

const char *ccut_kernel_name(uint32_t kid) {
  static const char *names[CCUT_K_COUNT] = {"affine_kernel", "sample_kernel", "hist_reduce_kernel",
                                            "exact_kernel", "sv_kernel", "parity_kernel",
                                            "transform_pass_kernel", "recombine_fp64_kernel",
                                            "zrecombine_fp64_kernel", "heisenberg_kernels",
                                            "mlp_kernels", "term_kernels", "carry_kernel"};
  return kid < CCUT_K_COUNT ? names[kid] : "";
}

}  // extern "C"

// ======================================================================
// Batches: many plans evaluated together.  The Clifford variants of all
// plans go through one persistent, work-queue tableau launch (tile shape
// picked by a small autotuner); everything else per plan follows; the whole
// sequence is captured once into a HIP graph and replayed.

struct ccut_batch {
  ccut_ctx *ctx = nullptr;
  std::vector<ccut_plan *> plans;
  std::vector<std::vector<uint32_t>> qubits;
  ccut_eval_opts eo{};
  Arena arena;
  std::vector<std::vector<char>> staged;
  hipStream_t stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool graphed = false;
  std::vector<double *> res;
  std::vector<FragDev> descs;
  std::vector<BatchItem> items;
  std::vector<std::vector<int64_t>> model_off;  // per plan, per fragment: word offset or -1
  uint64_t model_words_total = 0;
  // the measured Paulis of every Clifford descriptor (host rows, all
  // descriptors back to back), their carry-back jobs, the descriptors with
  // the carry-back stream, and each descriptor's row width
  std::vector<uint64_t> carry_rows;
  std::vector<CarryJob> carry_jobs;
  std::vector<FragDev> back_descs;
  std::vector<uint32_t> desc_w;
  uint32_t max_rows = 0;
  // independent per-plan steps run on a pool of streams (default priority),
  // forked from and joined back into the batch stream
  std::vector<hipStream_t> pool;
  hipEvent_t fork_ev = nullptr;
  std::vector<hipEvent_t> join_ev;
  // batched sampling and state vectors across plans: (plan, fragment) lists,
  // the non-Clifford descriptors and their state-vector shapes
  struct Ref {
    uint32_t plan, frag, desc, n_meas;
  };
  std::vector<Ref> samp;  // sampled Clifford fragments (desc indexes descs)
  std::vector<Ref> nc;    // non-Clifford fragments (desc indexes sv_descs)
  std::vector<FragDev> sv_descs;
  uint32_t max_m = 0, block = 64, grid = 0, tune_cached = 0;
  double tuned_ms = 0.0;
  // device outputs: the copy list of the last run (pinned and on the
  // device), reused while the caller passes the same output addresses, and
  // the event the caller's stream waits on
  std::vector<double *> last_outs;
  OutCopy *h_copy = nullptr, *d_copy = nullptr;
  hipEvent_t done_ev = nullptr;
  // the contraction jobs read their output address from out_tab[i] when
  // they run: res[i] while enqueuing eagerly; in a replay of the captured
  // graph the caller's device output itself, so no gather copies it
  // (job_out[i]: plan i's result comes from such a job, else from a launch
  // of its own into res[i])
  double **d_out_tab = nullptr, **h_out_tab = nullptr;
  std::vector<double *> cur_tab;
  std::vector<uint8_t> job_out;
  bool capturing = false;
  // durations of the state-vector classes (by their widest width) and of
  // the contraction classes (kCtrKey + class) measured in the creation run,
  // in ms; later enqueues place the classes on the streams by them
  struct Span {
    uint32_t key;
    hipEvent_t e0, e1;
  };
  std::vector<Span> spans;
  std::map<uint32_t, double> class_ms;
  bool measured = false;
  ~ccut_batch() {
    if (h_copy) (void)hipHostFree(h_copy);
    if (d_copy) (void)hipFree(d_copy);
    if (h_out_tab) (void)hipHostFree(h_out_tab);
    if (d_out_tab) (void)hipFree(d_out_tab);
    if (done_ev) (void)hipEventDestroy(done_ev);
    for (const Span &sp : spans) {
      (void)hipEventDestroy(sp.e0);
      (void)hipEventDestroy(sp.e1);
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (auto ps : pool) (void)hipStreamDestroy(ps);
    for (auto e : join_ev) (void)hipEventDestroy(e);
    if (fork_ev) (void)hipEventDestroy(fork_ev);
    if (stream) (void)hipStreamDestroy(stream);
    arena.release();
  }
};

namespace {

// Swap the context's execution state for the batch's while enqueueing.
struct BatchScope {
  ccut_ctx *c;
  ccut_batch *b;
  hipStream_t saved_stream;
  bool saved_timing, saved_aux;
  // timing: keep kernel timing on (eager runs only; a capture records no events)
  BatchScope(ccut_batch *bb, bool timing = false) : c(bb->ctx), b(bb) {
    std::swap(c->arena, b->arena);
    std::swap(c->staged, b->staged);
    saved_stream = c->stream;
    saved_timing = c->timing;
    saved_aux = c->use_aux;
    c->stream = c->cur = b->stream;
    c->timing = timing && saved_timing;
    c->use_aux = false;
  }
  ~BatchScope() {
    std::swap(c->arena, b->arena);
    std::swap(c->staged, b->staged);
    c->stream = c->cur = saved_stream;
    c->timing = saved_timing;
    c->use_aux = saved_aux;
    c->replay_uploads = false;
  }
};

// The affine sample models of every Clifford variant of the batch: one
// wave per item (grid-stride over the cost-sorted items) from the carried-back
// measured Paulis.
ccut_status batch_models(ccut_batch *b, FragDev *d_descs, const uint32_t *d_w, BatchItem *d_items,
                         const uint64_t *d_rows, uint64_t *d_models, uint32_t block, uint32_t grid) {
  ccut_ctx *c = b->ctx;
  if (b->items.empty()) return CCUT_OK;
  KTimer t(c, CCUT_K_AFFINE);
  HIP_TRY(c, launch_affine_batch(d_descs, d_w, d_items, (uint32_t)b->items.size(), d_rows, d_models, block, grid,
                                 c->cur));
  return CCUT_OK;
}

// Every Clifford descriptor's measured Paulis carried back through its
// fragment: one launch, one wave per descriptor.
ccut_status batch_carry(ccut_batch *b, uint64_t **d_rows_out) {
  ccut_ctx *c = b->ctx;
  *d_rows_out = nullptr;
  if (b->descs.empty()) return CCUT_OK;
  uint64_t *d_in = (uint64_t *)upload(c, b->carry_rows.data(), std::max<size_t>(b->carry_rows.size(), 1) * 8);
  uint64_t *d_out = aget<uint64_t>(c, std::max<size_t>(b->carry_rows.size(), 1));
  FragDev *d_back = (FragDev *)upload(c, b->back_descs.data(), b->back_descs.size() * sizeof(FragDev));
  CarryJob *d_jobs = (CarryJob *)upload(c, b->carry_jobs.data(), b->carry_jobs.size() * sizeof(CarryJob));
  if (!d_in || !d_out || !d_back || !d_jobs) return fail(c, CCUT_E_OOM, "device allocation failed");
  {
    KTimer t(c, CCUT_K_CARRY);
    HIP_TRY(c, launch_carry_batch(d_back, d_jobs, (uint32_t)b->carry_jobs.size(), b->max_m, b->max_rows, d_in, d_out,
                                  c->cur));
  }
  *d_rows_out = d_out;
  return CCUT_OK;
}

// Launch shapes of the affine-model launch chosen by timing, kept for the
// process (and, when CCUT_TUNE_CACHE names a file, across processes: one
// "key block per_cu ms" line per entry, read at the first lookup, appended
// when a new shape is tuned).  The key is the device (architecture, compute
// units) and the batch's model work: its item count and total elimination
// cost (sum of measurements^2 x row words), each bucketed by half octaves.
struct TuneEntry {
  uint32_t block, per_cu;
  double ms;
};
std::mutex g_tune_mu;
std::map<std::string, TuneEntry> g_tune;
bool g_tune_loaded = false;

std::string tune_key(ccut_ctx *c, const ccut_batch *b);
bool tune_lookup(const std::string &key, TuneEntry &e) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (!g_tune_loaded) {
    g_tune_loaded = true;
    if (const char *path = std::getenv("CCUT_TUNE_CACHE")) {
      if (FILE *f = std::fopen(path, "r")) {
        char k[256];
        unsigned blk = 0, pc = 0;
        double ms = 0.0;
        while (std::fscanf(f, "%255s %u %u %lf", k, &blk, &pc, &ms) == 4)
          if (blk && pc) g_tune[k] = TuneEntry{blk, pc, ms};
        std::fclose(f);
      }
    }
  }
  auto it = g_tune.find(key);
  if (it == g_tune.end()) return false;
  e = it->second;
  return true;
}
void tune_store(const std::string &key, const TuneEntry &e) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[key] = e;
  if (const char *path = std::getenv("CCUT_TUNE_CACHE")) {
    if (FILE *f = std::fopen(path, "a")) {
      std::fprintf(f, "%s %u %u %.6f\n", key.c_str(), e.block, e.per_cu, e.ms);
      std::fclose(f);
    }
  }
}

// Enqueue one whole batch evaluation on the batch stream (inside a
// BatchScope).  Allocation order is fixed, so a replay reuses the same memory.
std::string tune_key(ccut_ctx *c, const ccut_batch *b) {
  hipDeviceProp_t prop{};
  (void)hipGetDeviceProperties(&prop, c->device);
  double cost = 0.0;
  for (const BatchItem &it : b->items) {
    const double nm = b->descs[it.desc].n_meas;
    cost += nm * nm * b->desc_w[it.desc];
  }
  auto bucket = [](double x) { return x > 0 ? (int)std::floor(2.0 * std::log2(x)) : -1; };
  char buf[256];
  std::snprintf(buf, sizeof(buf), "%s:%d:%d:%d", prop.gcnArchName, prop.multiProcessorCount,
                bucket((double)b->items.size()), bucket(cost));
  for (char *p = buf; *p; ++p)
    if (*p == ' ') *p = '_';
  return buf;
}

constexpr uint32_t kCtrKey = 1u << 20;  // contraction classes' keys in the measured durations (above any width)

ccut_status batch_enqueue(ccut_batch *b, bool tune) {
  ccut_ctx *c = b->ctx;
  ccut_status st;
  // the creation run times its launches (events around them on their streams)
  auto span_begin = [&](uint32_t key, hipStream_t sm) -> int {
    if (!tune) return -1;
    ccut_batch::Span sp{key, nullptr, nullptr};
    if (hipEventCreate(&sp.e0) != hipSuccess) return -1;
    if (hipEventCreate(&sp.e1) != hipSuccess) {
      (void)hipEventDestroy(sp.e0);
      return -1;
    }
    b->spans.push_back(sp);
    (void)hipEventRecord(sp.e0, sm);
    return (int)b->spans.size() - 1;
  };
  auto span_end = [&](int i, hipStream_t sm) {
    if (i >= 0) (void)hipEventRecord(b->spans[(size_t)i].e1, sm);
  };
  c->arena.reset();
  if (!c->replay_uploads) c->staged.clear();
  // (an all-Heisenberg batch has no tableau items: allocate a placeholder, copy nothing)
  FragDev *d_descs = (FragDev *)upload(c, b->descs.empty() ? nullptr : b->descs.data(),
                                       std::max<size_t>(b->descs.size(), 1) * sizeof(FragDev));
  BatchItem *d_items = (BatchItem *)upload(c, b->items.empty() ? nullptr : b->items.data(),
                                           std::max<size_t>(b->items.size(), 1) * sizeof(BatchItem));
  uint32_t *d_w = (uint32_t *)upload(c, b->desc_w.empty() ? nullptr : b->desc_w.data(),
                                     std::max<size_t>(b->desc_w.size(), 1) * sizeof(uint32_t));
  uint64_t *d_models = aget<uint64_t>(c, std::max<uint64_t>(b->model_words_total, 1));
  if (!d_descs || !d_items || !d_w || !d_models) return fail(c, CCUT_E_OOM, "device allocation failed");
  // every plan's sampled outcome tables come from one pass of sampling
  // launches (plus one reduction), every non-Clifford fragment's from one
  // state-vector launch per shape; the per-plan steps below start from these
  // tables.  The state vectors need no tableau: they start at once, each
  // shape class on a pool stream of its own (at most 3 of them: HIP maps a
  // process's streams onto 4 hardware queues, the batch stream holds one),
  // and join before the per-plan steps.
  std::vector<std::vector<double *>> pre_dist(b->plans.size());
  std::vector<std::vector<uint16_t *>> pre_cnt(b->plans.size());  // sampled tables kept as 16-bit counts
  for (size_t i = 0; i < b->plans.size(); ++i) {
    pre_dist[i].assign(b->plans[i]->pd.frags.size(), nullptr);
    pre_cnt[i].assign(b->plans[i]->pd.frags.size(), nullptr);
  }
  const size_t n_sv_streams = std::min<size_t>(b->pool.size(), 3);
  std::vector<uint8_t> sv_used(n_sv_streams, 0);
  // the descriptors' copy goes on the batch stream ahead of the fork point
  // the state-vector streams wait for
  FragDev *d_sv = nullptr;
  if (!b->nc.empty()) {
    d_sv = (FragDev *)upload(c, b->sv_descs.data(), b->sv_descs.size() * sizeof(FragDev));
    if (!d_sv) return fail(c, CCUT_E_OOM, "device allocation failed");
  }
  // the state-vector classes, their tables and their job lists, uploaded in
  // the classes' fixed order on the batch stream ahead of the fork point
  // (the launches come later, on the pool streams, in the order of their
  // durations)
  struct SvClass {
    uint32_t m;
    std::vector<SvJob> jobs[2];
    SvJob *d_jobs[2] = {nullptr, nullptr};
    uint64_t wg[2] = {0, 0};
    size_t lds[2] = {0, 0};
    double cost = 0.0;
  };
  // one class per launch shape (register and wave bits): every state of
  // up to 8 qubits shares one; C.m is the class's widest state
  std::vector<SvClass> classes;
  auto shape_key = [](uint32_t m) {
    const SvShape sh = sv_shape(m);
    return sh.rb * 64u + sh.wb;
  };
  for (uint32_t m = 1; m <= (uint32_t)kMaxNcQubits; ++m) {
    if (m > 1 && shape_key(m - 1) == shape_key(m)) continue;  // handled with the class's first width
    SvClass C;
    C.m = m;
    for (const auto &ref : b->nc) {
      const FragDev &h = b->sv_descs[ref.desc];
      if (shape_key(h.m) != shape_key(m)) continue;
      C.m = std::max(C.m, h.m);
      double *dist = aget<double>(c, h.n_variants << ref.n_meas);
      const size_t sb = sv_states_bytes(h);
      double *states = sb ? aget<double>(c, sb / sizeof(double)) : nullptr;
      if (!dist || (sb && !states)) return fail(c, CCUT_E_OOM, "device allocation failed");
      pre_dist[ref.plan][ref.frag] = dist;
      const uint32_t passes[2] = {sb ? 1u : 0u, 2u};
      for (int k = 0; k < (sb ? 2 : 1); ++k) {
        uint64_t n_wg;
        uint32_t bs;
        size_t l;
        bool split;
        sv_pass_shape(h, passes[k], n_wg, bs, l, split);
        SvJob J{};
        J.desc = ref.desc;
        J.split = split ? 1u : 0u;
        J.wg0 = C.wg[k];
        J.dist = dist;
        J.mode = passes[k];
        J.states = states;
        C.wg[k] += n_wg;
        C.lds[k] = std::max(C.lds[k], l);
        C.cost += (double)n_wg * (double)(1u << h.m) * (passes[k] == 2 ? 8.0 : (double)h.n_ops);
        C.jobs[k].push_back(J);
      }
    }
    if (!C.jobs[0].empty()) classes.push_back(std::move(C));
  }
  // the job lists go up in the classes' fixed order (a re-enqueue reuses
  // the first run's uploads in place: the order must not depend on the
  // launch order below)
  for (SvClass &C : classes)
    for (int k = 0; k < 2; ++k) {
      if (C.jobs[k].empty()) continue;
      C.d_jobs[k] = (SvJob *)upload(c, C.jobs[k].data(), C.jobs[k].size() * sizeof(SvJob));
      if (!C.d_jobs[k]) return fail(c, CCUT_E_OOM, "device allocation failed");
    }
  if (!b->nc.empty() && n_sv_streams) HIP_TRY(c, hipEventRecord(b->fork_ev, b->stream));
  auto sv_pass = [&]() -> ccut_status {
    if (!b->nc.empty()) {
      // (the fork point was recorded before the sampling chain)
      for (size_t k = 0; k < n_sv_streams; ++k) HIP_TRY(c, hipStreamWaitEvent(b->pool[k], b->fork_ev, 0));
      // two launches per shape class: the first runs fragments without
      // quantum inputs in full and evolves the computational-basis inputs of
      // the others, the second combines those into their preparations; the
      // classes go to the streams longest first, each to the stream with the
      // least work so far (work: amplitudes times program length, summed over
      // workgroups)
      // measured durations (ms) replace the estimates once the creation run has timed the classes
      if (b->measured)
        for (SvClass &C : classes) {
          auto it = b->class_ms.find(C.m);
          if (it != b->class_ms.end()) C.cost = it->second;
        }
      std::stable_sort(classes.begin(), classes.end(),
                       [](const SvClass &x, const SvClass &y) { return x.cost > y.cost; });
      std::vector<double> load(n_sv_streams, 0.0);
      for (const SvClass &C : classes) {
        if (n_sv_streams) {
          const size_t k = (size_t)(std::min_element(load.begin(), load.end()) - load.begin());
          load[k] += C.cost;
          c->cur = b->pool[k];
          sv_used[k] = 1;
        }
        const int sp = span_begin(C.m, c->cur);
        for (int k = 0; k < 2; ++k) {
          if (C.jobs[k].empty()) continue;
          KTimer tm(c, CCUT_K_SV);
          HIP_TRY(c, launch_sv_batch(d_sv, C.d_jobs[k], (uint32_t)C.jobs[k].size(), C.wg[k], C.m, C.lds[k], c->cur));
        }
        span_end(sp, c->cur);
      }
      c->cur = b->stream;
      for (size_t k = 0; k < n_sv_streams; ++k)
        if (sv_used[k]) HIP_TRY(c, hipEventRecord(b->join_ev[k], b->pool[k]));
    }
    return CCUT_OK;
  };
  uint64_t *d_rows = nullptr;
  if ((st = batch_carry(b, &d_rows)) != CCUT_OK) return st;
  TuneEntry cached{};
  std::string tkey;
  bool time_models = tune;  // the creation run times the model launch's candidates, unless cached
  if (tune && !b->items.empty()) {
    tkey = tune_key(c, b);
    if (tune_lookup(tkey, cached)) {
      int cus = 256;
      (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device);
      const uint64_t full = (b->items.size() * 64 + cached.block - 1) / cached.block;
      b->block = cached.block;
      b->grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(full, (uint64_t)cus * cached.per_cu));
      b->tuned_ms = cached.ms;
      b->tune_cached = 1;
      time_models = false;
    }
  }
  if (time_models && !b->items.empty()) {
    // autotune the model launch: waves per workgroup x workgroups per
    // compute unit (a grid-stride loop covers whatever the grid leaves)
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device);
    uint32_t best_pc = 1;
    hipEvent_t e0, e1;
    HIP_TRY(c, hipEventCreate(&e0));
    HIP_TRY(c, hipEventCreate(&e1));
    double best = 1e30;
    const uint64_t n_items = b->items.size();
    for (uint32_t block : {64u, 256u, 1024u}) {
      const uint64_t full = (n_items * 64 + block - 1) / block;
      for (uint32_t per_cu : {1u, 2u, 4u, 8u, 32u}) {
        const uint32_t grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(full, (uint64_t)cus * per_cu));
        // warm once, then time
        if ((st = batch_models(b, d_descs, d_w, d_items, d_rows, d_models, block, grid)) != CCUT_OK) return st;
        HIP_TRY(c, hipEventRecord(e0, c->cur));
        if ((st = batch_models(b, d_descs, d_w, d_items, d_rows, d_models, block, grid)) != CCUT_OK) return st;
        HIP_TRY(c, hipEventRecord(e1, c->cur));
        HIP_TRY(c, hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_TRY(c, hipEventElapsedTime(&ms, e0, e1));
        if (ms < best) {
          best = ms;
          b->block = block;
          b->grid = grid;
          best_pc = per_cu;
        }
        if (grid == full) break;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->tuned_ms = best;
    tune_store(tkey, TuneEntry{b->block, best_pc, best});
  }
  if ((st = batch_models(b, d_descs, d_w, d_items, d_rows, d_models, b->block, b->grid)) != CCUT_OK) return st;
  if (!b->samp.empty()) {
    // jobs in LDS classes (one launch each, so a launch's workgroups reserve
    // only their class's histogram): up to 20 KiB (eight workgroups per CU,
    // as many as the wave slots allow, so one class), 40, 72 and 136 KiB
    constexpr int kClasses = 4;
    const uint64_t shots = b->eo.shots_per_variant;
    const uint64_t nquads = (shots + 3) / 4;
    auto lds_class = [](size_t l) {
      return l <= (20u << 10) ? 0 : l <= (40u << 10) ? 1 : l <= (72u << 10) ? 2 : 3;
    };
    auto sliced_bits = [](uint32_t nm) { return nm > kLdsHistBits && nm <= kLdsHistBits + kMaxSliceBits; };
    std::vector<size_t> order;
    for (int cls = 0; cls < kClasses; ++cls)
      for (size_t q = 0; q < b->samp.size(); ++q)
        if (lds_class(sample_lds_bytes(b->samp[q].n_meas, true, sliced_bits(b->samp[q].n_meas))) == cls)
          order.push_back(q);
    std::vector<SampleJob> jobs;
    uint64_t t = 0, fill_words = 0;
    uint64_t cls_units[kClasses] = {};
    size_t cls_lds[kClasses] = {}, cls_first[kClasses] = {}, cls_count[kClasses] = {};
    for (size_t q : order) {
      const auto &ref = b->samp[q];
      const FragDev &h = b->descs[ref.desc];
      const uint32_t nm = ref.n_meas, bins = 1u << nm;
      const uint64_t nv = h.n_variants;
      // up to 3 bits above the LDS histogram: one workgroup per 2^14-bin
      // slice, each replaying the shots (no global atomics, no zero fill)
      const uint32_t nslice = sliced_bits(nm) ? 1u << (nm - kLdsHistBits) : 1u;
      const bool lds = nm <= kLdsHistBits || nslice > 1;
      uint32_t nblk;
      if (lds) {  // 16384 shots or more per block: a batch has workgroups enough without splitting further
        const uint64_t per_block = std::max<uint64_t>(std::min<uint64_t>(bins, 1u << kLdsHistBits), 16384);
        nblk = (uint32_t)std::max<uint64_t>(1, std::min((shots + per_block - 1) / per_block, (nquads + kSampleThreads - 1) / kSampleThreads));
        // and few enough for the 16-bit LDS counts
        nblk = (uint32_t)std::max<uint64_t>(nblk, (nquads + kMaxUnitQpt * kSampleThreads - 1) / (kMaxUnitQpt * kSampleThreads));
      } else {
        nblk = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((nquads + 1023) / 1024, 4096));
        fill_words += nv * (uint64_t)bins;
      }
      const size_t lds_need = sample_lds_bytes(nm, true, nslice > 1);
      const int cls = lds_class(lds_need);
      if (cls_count[cls]++ == 0) cls_first[cls] = jobs.size();
      cls_lds[cls] = std::max<size_t>(cls_lds[cls], lds_need);
      SampleJob J{};
      J.models = d_models + b->model_off[ref.plan][ref.frag];
      J.shots = shots;
      J.seed = b->eo.seed;
      J.vid0 = h.vid_base;
      J.nv = nv;
      J.n_meas = nm;
      J.nblk = nblk;
      J.qpt = (uint32_t)((nquads + (uint64_t)nblk * kSampleThreads - 1) / ((uint64_t)nblk * kSampleThreads));
      J.nslice = nslice;
      J.wg0 = cls_units[cls];
      J.rb0 = t;
      cls_units[cls] += nv * nblk * nslice;
      // one shot block in LDS: the sampling workgroups write the table
      // themselves; otherwise partial counts and a reduction
      if (!(lds && nblk == 1)) t += (nv * bins + 4095) / 4096;  // reduction workgroups
      jobs.push_back(J);
    }
    // partial counts: the per-variant ones (zeroed) first, contiguous
    uint32_t *zeroed = fill_words ? aget<uint32_t>(c, fill_words) : nullptr;
    if (fill_words && !zeroed) return fail(c, CCUT_E_OOM, "device allocation failed");
    uint64_t zo = 0;
    for (size_t q = 0; q < jobs.size(); ++q) {
      SampleJob &J = jobs[q];
      const uint64_t bins = 1ull << J.n_meas;
      if ((J.n_meas <= kLdsHistBits || J.nslice > 1) && J.nblk == 1) {
        J.partial = nullptr;  // written directly as the table
      } else if (J.n_meas <= kLdsHistBits || J.nslice > 1) {
        J.partial = aget<uint32_t>(c, J.nv * J.nblk * bins);
      } else {
        J.partial = zeroed + zo;
        zo += J.nv * bins;
      }
      // 16-bit shot counts where the consumer reads them: the fold target of
      // a matrix-path contraction, or a fragment that goes through the tiled
      // transform
      const auto &ref = b->samp[order[q]];
      bool c16 = false;
      if (J.shots <= 0xFFFFull) {
        ccut_plan *pp = b->plans[ref.plan];
        const uint32_t *qb = b->qubits[ref.plan].data();
        const uint32_t nqb = (uint32_t)b->qubits[ref.plan].size();
        const Fragment &fr = pp->pd.frags[ref.frag];
        ccut_eval_opts eo_i = b->eo;
        if (fold_target(pp->pd, &eo_i, qb, nqb) == (int)ref.frag) {
          c16 = counts_contraction(pp->pd, &eo_i, nqb);
        } else {
          const FragRequest rr = marginal_request(fr, qb, nqb);
          TileJob probe;
          c16 = !fr.axes.empty() && tile_job(fr, rr, nullptr, 1ull << rr.meas.size(), nullptr, probe);
        }
      }
      if (c16) {
        J.cnt16 = aget<uint16_t>(c, J.nv * bins);
        J.dist = nullptr;
      } else {
        J.dist = aget<double>(c, J.nv * bins);
      }
      if ((!J.partial && J.nblk != 1) || (!J.dist && !J.cnt16)) return fail(c, CCUT_E_OOM, "device allocation failed");
      pre_dist[ref.plan][ref.frag] = J.dist;
      pre_cnt[ref.plan][ref.frag] = J.cnt16;
    }
    SampleJob *d_jobs = (SampleJob *)upload(c, jobs.data(), jobs.size() * sizeof(SampleJob));
    if (!d_jobs) return fail(c, CCUT_E_OOM, "device allocation failed");
    if (fill_words) HIP_TRY(c, launch_fill_u32(zeroed, fill_words, 0u, c->cur));
    // every class on the batch stream, one after another: the classes are
    // throughput-bound, and spread over the pool streams beside the state
    // vectors they only slowed each other down (measured)
    for (int cls = 0; cls < kClasses; ++cls)
      if (cls_count[cls]) {
        KTimer tm(c, CCUT_K_SAMPLE);
        HIP_TRY(c, launch_sample_batch(d_jobs + cls_first[cls], (uint32_t)cls_count[cls], cls_units[cls],
                                       cls_lds[cls], c->cur));
      }
    if (t) {
      KTimer tm(c, CCUT_K_HIST_REDUCE);
      HIP_TRY(c, launch_hist_reduce_batch(d_jobs, (uint32_t)jobs.size(), t, c->cur));
    }
  }
  // the state vectors (pool streams; their job lists went up before the fork
  // point), enqueued after the sampling chain: a graph replay starts its
  // nodes in capture order, and the chain is the longer of the two
  if ((st = sv_pass()) != CCUT_OK) return st;
  for (size_t k = 0; k < n_sv_streams; ++k)
    if (sv_used[k]) HIP_TRY(c, hipStreamWaitEvent(b->stream, b->join_ev[k], 0));
  // The plans' remaining steps.  Work that the batched launches below do
  // not cover (Heisenberg tensors, tables outside the pre-pass, transforms
  // too large to tile, contractions of more than 8 fragments) runs per plan,
  // plan i on pool stream i mod P; then, on the batch stream, one tiled
  // transform launch for every other fragment, one plain and one MFMA
  // contraction launch for all plans.  Each plan takes the same transform
  // and contraction as a call of its own, so the results are the same bits.
  const size_t P = b->pool.size(), np = b->plans.size();
  HIP_TRY(c, hipEventRecord(b->fork_ev, b->stream));
  for (size_t k = 0; k < P; ++k) HIP_TRY(c, hipStreamWaitEvent(b->pool[k], b->fork_ev, 0));
  const bool fp32 = b->eo.precision != CCUT_FP64;
  std::vector<TileJob> tjobs;
  std::vector<FoldJob> fjobs;
  std::vector<RecombArgs> rargs(np);
  std::vector<uint8_t> kind(np);  // 0 plain (batched), 1 plain (own launch), 2 MFMA
  for (size_t i = 0; i < np; ++i) {
    ccut_plan *p = b->plans[i];
    const PlanData &pd = p->pd;
    if (pd.frags.size() > (size_t)kMaxFrags) return fail(c, CCUT_E_UNSUPPORTED, "more than 64 fragments");
    ccut_eval_opts eo = b->eo;
    eo.circuit = (uint32_t)i;
    const uint32_t *qubits = b->qubits[i].data();
    const uint32_t nq = (uint32_t)b->qubits[i].size();
    double *res = aget<double>(c, (size_t)1 << nq);
    if (!res) return fail(c, CCUT_E_OOM, "device allocation failed");
    if (b->res.size() <= i) b->res.push_back(res);
    b->res[i] = res;
    RecombArgs &args = rargs[i];
    args = RecombArgs{};
    args.n_frags = (uint32_t)pd.frags.size();
    args.k = pd.k;
    args.lo_parts = b->eo.precision == CCUT_FP32X3_MFMA_FP64SUM;
    c->stream = c->cur = P ? b->pool[i % P] : b->stream;
    const int g = fold_target(pd, &eo, qubits, nq);
    std::vector<char> folded(pd.frags.size(), 0);
    for (const Fragment &f : pd.frags) {
      FragRequest r = marginal_request(f, qubits, nq);
      double *T = nullptr;
      if (use_heisenberg(f, &eo, r.req_pos.size())) {
        st = heis_tensor(p, f, r, eo.circuit, nullptr, &T);
      } else {
        double *dist = pre_dist[i][f.index];
        uint16_t *cnt = pre_cnt[i][f.index];
        uint64_t *pm = b->model_off[i][f.index] >= 0 ? d_models + b->model_off[i][f.index] : nullptr;
        st = (dist || cnt) ? CCUT_OK : variant_dists(p, &eo, f, r, &dist, pm);
        const uint64_t xsize = 1ull << r.meas.size();
        TileJob J;
        if (st == CCUT_OK && (int)f.index == g) {
          // tables [preparations][outcomes] stand in for the tensor (fold_target)
          T = cnt ? reinterpret_cast<double *>(cnt) : dist;
          if (cnt) {
            args.f[f.index].cnt16 = 1;
            args.f[f.index].shots = (double)eo.shots_per_variant;
          }
        } else if (st == CCUT_OK && !f.axes.empty() && tile_job(f, r, dist, xsize, nullptr, J)) {
          J.in16 = cnt;
          J.shots = (double)eo.shots_per_variant;
          J.fold = fold_mask(pd, g, f);  // the fold of fold_jobs, applied in the tile
          folded[f.index] = 1;
          J.out = T = aget<double>(c, J.x_out << (2 * f.axes.size()));
          if (!T) st = fail(c, CCUT_E_OOM, "device allocation failed");
          tjobs.push_back(J);
        } else if (st == CCUT_OK) {
          st = pauli_passes(c, f, r, dist, xsize, 0, &T);
        }
      }
      if (st != CCUT_OK) break;
      RecombFrag &rf = args.f[f.index];
      rf.T = T;
      rf.n_axes = (uint32_t)f.axes.size();
      rf.rows = 1u << r.req_pos.size();
      rf.n_req = (uint32_t)r.req_pos.size();
      for (size_t j = 0; j < f.axes.size(); ++j) rf.axis_cut[j] = f.axes[j].cut;
      for (size_t q = 0; q < r.req_user.size(); ++q) rf.req_user[q] = r.req_user[q];
    }
    c->stream = c->cur = b->stream;
    if (st != CCUT_OK) return st;
    fold_jobs(pd, g, args, fjobs, &folded);
    // the contraction recombine() would take
    const uint64_t K = 1ull << (2 * pd.k);
    kind[i] = plain_contraction(args, nq, fp32) ? (args.n_frags <= 8 ? 0 : 1) : 2;
  }
  for (size_t k = 0; k < P; ++k) {
    HIP_TRY(c, hipEventRecord(b->join_ev[k], b->pool[k]));
    HIP_TRY(c, hipStreamWaitEvent(b->stream, b->join_ev[k], 0));
  }
  if (!tjobs.empty()) {
    uint64_t wg = 0;
    for (TileJob &J : tjobs) {
      J.wg0 = wg;
      wg += J.tiles;
    }
    TileJob *d_t = (TileJob *)upload(c, tjobs.data(), tjobs.size() * sizeof(TileJob));
    if (!d_t) return fail(c, CCUT_E_OOM, "device allocation failed");
    KTimer t(c, CCUT_K_TRANSFORM);
    HIP_TRY(c, launch_transform_tiled(d_t, (uint32_t)tjobs.size(), wg, c->cur));
  }
  if (!fjobs.empty()) {
    FoldJob *d_fj = (FoldJob *)upload(c, fjobs.data(), fjobs.size() * sizeof(FoldJob));
    if (!d_fj) return fail(c, CCUT_E_OOM, "device allocation failed");
    KTimer t(c, CCUT_K_TRANSFORM);
    HIP_TRY(c, launch_fold(d_fj, (uint32_t)fjobs.size(), c->cur));
  }
  // the output table: res while enqueuing eagerly; a captured graph reads
  // whatever the run call has put there
  b->job_out.assign(np, 0);
  for (size_t i = 0; i < np; ++i) b->job_out[i] = kind[i] != 1;
  if (!b->capturing && b->cur_tab != b->res) {
    HIP_TRY(c, hipStreamSynchronize(b->stream));  // an earlier copy may still read the pinned table
    for (size_t i = 0; i < np; ++i) b->h_out_tab[i] = b->res[i];
    HIP_TRY(c, hipMemcpyAsync(b->d_out_tab, b->h_out_tab, np * sizeof(double *), hipMemcpyHostToDevice, b->stream));
    b->cur_tab = b->res;
  }
  // contractions: the plain ones' arguments in one upload, the MFMA ones'
  // operand descriptions in another
  std::vector<RecombArgs> plain;
  std::vector<size_t> plain_of(np, 0);
  std::vector<GemmArgs> gargs;
  for (size_t i = 0; i < np; ++i) {
    if (kind[i] < 2) {
      plain_of[i] = plain.size();
      plain.push_back(rargs[i]);
    } else {
      gargs.emplace_back();
      make_gemm_args(rargs[i], gargs.back());
    }
  }
  RecombArgs *d_plain = plain.empty() ? nullptr : (RecombArgs *)upload(c, plain.data(), plain.size() * sizeof(RecombArgs));
  GemmArgs *d_gargs = gargs.empty() ? nullptr : (GemmArgs *)upload(c, gargs.data(), gargs.size() * sizeof(GemmArgs));
  if ((!plain.empty() && !d_plain) || (!gargs.empty() && !d_gargs)) return fail(c, CCUT_E_OOM, "device allocation failed");
  std::vector<RcJob> rjobs;
  // launch classes: 0 the MFMA tiles, 1 + 3 log2(M) + log2(CPT) the skinny
  // kernel for M rows and CPT columns per thread
  constexpr int kGemmClasses = 19;
  std::vector<GemmJob> gjobs[kGemmClasses];
  uint64_t rwg = 0, gwg[kGemmClasses] = {}, grwg[kGemmClasses] = {};
  bool ggen[kGemmClasses] = {};
  size_t glds[kGemmClasses] = {};
  for (size_t i = 0, g = 0; i < np; ++i) {
    const uint32_t nq = (uint32_t)b->qubits[i].size();
    if (kind[i] == 0) {
      RcJob J{};
      J.args = d_plain + plain_of[i];
      J.out = b->d_out_tab + i;
      J.nq = nq;
      J.wg0 = rwg;
      rwg += ((1ull << nq) + kRcChunkOut - 1) / kRcChunkOut;
      rjobs.push_back(J);
    } else if (kind[i] == 2) {
      const GemmArgs &h = gargs[g];
      const bool skinny = contraction_skinny(h, fp32);
      int sk = 0;
      if (skinny) {
        int lm = 0, lc = 0;
        while ((1u << lm) < h.M) ++lm;
        while ((1u << lc) < skinny_cols(h)) ++lc;
        sk = 1 + 3 * lm + lc;
      }
      GemmJob J{};
      J.args = d_gargs + g;
      J.splits = contraction_splits(h, skinny);
      J.tiles = gemm_tiles(h, skinny);
      J.k_per_split = gemm_k_per_split(h, J.splits, skinny);
      const bool direct = J.splits == 1;  // one split: the kernel writes the outputs itself
      J.partial = direct ? nullptr : aget<double>(c, (size_t)J.splits * h.M * h.N);
      if (!direct && !J.partial) return fail(c, CCUT_E_OOM, "device allocation failed");
      J.out = b->d_out_tab + i;
      J.wg0 = gwg[sk];
      J.rwg0 = grwg[sk];
      gwg[sk] += (uint64_t)J.tiles * J.splits;
      if (!skinny) {
        ggen[sk] = ggen[sk] || gemm_general(h);
        glds[sk] = std::max(glds[sk], gemm_fac_lds(h));
      }
      if (!direct) grwg[sk] += ((uint64_t)h.M * h.N + 255) / 256;
      gjobs[sk].push_back(J);
      ++g;
    }
  }
  // every job list goes up on the batch stream first; then the launch
  // classes (they write disjoint outputs and partial sums) spread over the
  // batch stream and up to three pool streams, which are idle by now, so the
  // small skinny classes run beside the large plain and MFMA launches
  RcJob *d_r = nullptr;
  if (!rjobs.empty() && !(d_r = (RcJob *)upload(c, rjobs.data(), rjobs.size() * sizeof(RcJob))))
    return fail(c, CCUT_E_OOM, "device allocation failed");
  GemmJob *d_g[kGemmClasses] = {};
  for (int sk = 0; sk < kGemmClasses; ++sk)
    if (!gjobs[sk].empty() &&
        !(d_g[sk] = (GemmJob *)upload(c, gjobs[sk].data(), gjobs[sk].size() * sizeof(GemmJob))))
      return fail(c, CCUT_E_OOM, "device allocation failed");
  const size_t n_side = std::min<size_t>(P, 3);
  if (n_side) {
    HIP_TRY(c, hipEventRecord(b->fork_ev, b->stream));
    for (size_t k = 0; k < n_side; ++k) HIP_TRY(c, hipStreamWaitEvent(b->pool[k], b->fork_ev, 0));
  }
  // the launch classes (-1: the plain sums, else the matrix class); the
  // creation run puts them round-robin on the streams and times them, later
  // enqueues place them longest first on the least-loaded stream
  std::vector<int> cls;
  if (!rjobs.empty()) cls.push_back(-1);
  for (int sk = 0; sk < kGemmClasses; ++sk)
    if (!gjobs[sk].empty()) cls.push_back(sk);
  const size_t n_str = n_side + 1;
  std::vector<size_t> where(cls.size()), seq(cls.size());
  for (size_t i = 0; i < cls.size(); ++i) {
    where[i] = i % n_str;
    seq[i] = i;
  }
  if (b->measured) {
    std::vector<double> cost(cls.size(), 0.0), load(n_str, 0.0);
    for (size_t i = 0; i < cls.size(); ++i) {
      auto it = b->class_ms.find(kCtrKey + (uint32_t)(cls[i] + 1));
      if (it != b->class_ms.end()) cost[i] = it->second;
    }
    std::stable_sort(seq.begin(), seq.end(), [&](size_t x, size_t y) { return cost[x] > cost[y]; });
    for (size_t i : seq) {
      const size_t k = (size_t)(std::min_element(load.begin(), load.end()) - load.begin());
      load[k] += cost[i];
      where[i] = k;
    }
  }
  for (size_t i : seq) {
    c->cur = where[i] ? b->pool[where[i] - 1] : b->stream;
    const int sk = cls[i];
    const int sp = span_begin(kCtrKey + (uint32_t)(sk + 1), c->cur);
    KTimer t(c, CCUT_K_RECOMBINE);
    if (sk < 0) {
      HIP_TRY(c, launch_recombine_batch(d_r, (uint32_t)rjobs.size(), rwg, c->cur));
    } else {
      const int mode = fp32 ? (b->eo.precision == CCUT_FP32X3_MFMA_FP64SUM ? 2 : 1) : 0;
      HIP_TRY(c, launch_gemm_batch(d_g[sk], (uint32_t)gjobs[sk].size(), gwg[sk], grwg[sk], mode, ggen[sk], glds[sk],
                                   sk ? 1u << ((sk - 1) / 3) : 0u, sk ? 1u << ((sk - 1) % 3) : 0u, c->cur));
    }
    span_end(sp, c->cur);
  }
  c->cur = b->stream;
  for (size_t k = 0; k < n_side; ++k) {
    HIP_TRY(c, hipEventRecord(b->join_ev[k], b->pool[k]));
    HIP_TRY(c, hipStreamWaitEvent(b->stream, b->join_ev[k], 0));
  }
  KTimer t(c, CCUT_K_RECOMBINE);
  for (size_t i = 0; i < np; ++i)
    if (kind[i] == 1)
      HIP_TRY(c, launch_recombine_fp64(d_plain + plain_of[i], rargs[i].n_frags, (uint32_t)b->qubits[i].size(),
                                       b->res[i], c->cur));
  return CCUT_OK;
}

}  // namespace

extern "C" {

ccut_status ccut_batch_create(ccut_ctx *c, ccut_plan *const *plans, size_t n, const ccut_eval_opts *eo,
                              const uint32_t *const *qubits, const uint32_t *nq, int use_graph, ccut_batch **out) {
  if (!c || !out || !eo || (n && (!plans || !qubits || !nq))) return fail(c, CCUT_E_INVALID, "NULL argument");
  *out = nullptr;
  if (c->device < 0) return fail(c, CCUT_E_DEVICE, "host-only context: evaluation needs a device");
  if (n == 0 || n > 65535) return fail(c, CCUT_E_INVALID, "batch size must be in [1, 65535]");
  if (eo->flags) return fail(c, CCUT_E_UNSUPPORTED, "evaluation flags apply to single calls");
  std::unique_ptr<ccut_batch> b(new (std::nothrow) ccut_batch());
  if (!b) return fail(c, CCUT_E_OOM, "host allocation failed");
  b->ctx = c;
  b->eo = *eo;
  b->arena.alloc = c->arena.alloc;
  b->arena.free_fn = c->arena.free_fn;
  b->arena.user = c->arena.user;
  ccut_status st;
  for (size_t i = 0; i < n; ++i) {
    ccut_plan *p = plans[i];
    if (!p || p->ctx != c) return fail(c, CCUT_E_INVALID, "plan from another context");
    if ((st = check_eval(p, eo)) != CCUT_OK) return st;
    if ((st = check_request(c, p->pd.n, qubits[i], nq[i])) != CCUT_OK) return st;
    b->plans.push_back(p);
    b->qubits.emplace_back(qubits[i], qubits[i] + nq[i]);
    std::vector<int64_t> offs(p->pd.frags.size(), -1);
    for (const Fragment &f : p->pd.frags) {
      if (!f.clifford) {
        FragRequest r = marginal_request(f, qubits[i], nq[i]);
        if (r.meas.size() > (size_t)kMaxTableBits)
          return fail(c, CCUT_E_UNSUPPORTED, "outcome table over more than 24 measured qubits");
        b->nc.push_back({(uint32_t)i, f.index, (uint32_t)b->sv_descs.size(), (uint32_t)r.meas.size()});
        b->sv_descs.push_back(frag_desc(p, f, r, (uint32_t)i));
        continue;
      }
      FragRequest r = marginal_request(f, qubits[i], nq[i]);
      if (use_heisenberg(f, eo, r.req_pos.size())) continue;
      const uint32_t nm = (uint32_t)r.meas.size();
      if (nm > (uint32_t)kMaxMeas) return fail(c, CCUT_E_UNSUPPORTED, "more than 64 measured qubits");
      if (f.m() > 512) return fail(c, CCUT_E_UNSUPPORTED, "Clifford fragment wider than 512 qubits");
      FragDev h = frag_desc(p, f, r, (uint32_t)i);
      const uint32_t di = (uint32_t)b->descs.size();
      if (di >= (1u << 28)) return fail(c, CCUT_E_UNSUPPORTED, "too many Clifford fragments in one batch");
      b->descs.push_back(h);
      const uint32_t Wb = row_words(f.m());
      const std::vector<uint64_t> rows = measured_rows(h, Wb);
      const uint64_t boff = b->carry_rows.size();
      const uint32_t n_rows = (uint32_t)(rows.size() / (2 * Wb + 1));
      b->carry_rows.insert(b->carry_rows.end(), rows.begin(), rows.end());
      b->carry_jobs.push_back({di, Wb, n_rows, 0u, boff, boff});
      FragDev hb = h;
      hb.ops = p->d_back[f.index];
      hb.n_ops = p->n_back[f.index];
      hb.layers = p->d_back_layers[f.index];
      hb.n_layers = p->n_back_layers[f.index];
      b->back_descs.push_back(hb);
      b->desc_w.push_back(Wb);
      b->max_rows = std::max(b->max_rows, n_rows);
      offs[f.index] = (int64_t)b->model_words_total;
      if (eo->shots_per_variant) {
        if (nm > (uint32_t)kMaxTableBits)
          return fail(c, CCUT_E_UNSUPPORTED, "outcome table over more than 24 measured qubits");
        b->samp.push_back({(uint32_t)i, f.index, di, nm});
      }
      for (uint64_t v = 0; v < f.n_variants; ++v)
        b->items.push_back({di, 0u, v, b->model_words_total + v * model_words(nm), boff});
      b->model_words_total += f.n_variants * model_words(nm);
      b->max_m = std::max(b->max_m, f.m());
    }
    b->model_off.push_back(offs);
  }
  // longest items first: the elimination costs ~ measurements^2 x row width
  std::stable_sort(b->items.begin(), b->items.end(), [&](const BatchItem &x, const BatchItem &y) {
    const FragDev &a = b->descs[x.desc], &d = b->descs[y.desc];
    return (uint64_t)a.n_meas * a.n_meas * b->desc_w[x.desc] > (uint64_t)d.n_meas * d.n_meas * b->desc_w[y.desc];
  });
  HIP_TRY(c, hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
  HIP_TRY(c, hipEventCreateWithFlags(&b->fork_ev, hipEventDisableTiming));
  HIP_TRY(c, hipMalloc((void **)&b->d_out_tab, std::max<size_t>(n, 1) * sizeof(double *)));
  HIP_TRY(c, hipHostMalloc((void **)&b->h_out_tab, std::max<size_t>(n, 1) * sizeof(double *), hipHostMallocDefault));
  for (size_t k = 0; k < std::min<size_t>(n, 8); ++k) {
    hipStream_t ps = nullptr;
    hipEvent_t je = nullptr;
    HIP_TRY(c, hipStreamCreateWithFlags(&ps, hipStreamNonBlocking));
    b->pool.push_back(ps);
    HIP_TRY(c, hipEventCreateWithFlags(&je, hipEventDisableTiming));
    b->join_ev.push_back(je);
  }
  {
    BatchScope scope(b.get());
    if ((st = batch_enqueue(b.get(), true)) != CCUT_OK) return st;
  }
  HIP_TRY(c, hipStreamSynchronize(b->stream));
  // the creation run's launch durations
  for (const ccut_batch::Span &sp : b->spans) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, sp.e0, sp.e1) != hipSuccess) continue;
    b->class_ms[sp.key] = ms;
  }
  (void)hipGetLastError();
  b->measured = !b->spans.empty();
  if (use_graph) {
    BatchScope scope(b.get());
    c->replay_uploads = true;
    hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      b->capturing = true;
      st = batch_enqueue(b.get(), false);
      b->capturing = false;
      hipGraph_t g = nullptr;
      e = hipStreamEndCapture(b->stream, &g);
      if (st == CCUT_OK && e == hipSuccess && g) {
        b->graph = g;
        if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) == hipSuccess) b->graphed = true;
      } else if (g) {
        (void)hipGraphDestroy(g);
      }
    }
    (void)hipGetLastError();
    c->err.clear();
  }
  *out = b.release();
  ctx_retain(c);
  return CCUT_OK;
}

ccut_status ccut_batch_run(ccut_batch *b, double *const *outs, int outs_on_device) {
  if (!b || !outs) return CCUT_E_INVALID;
  ccut_ctx *c = b->ctx;
  HIP_TRY(c, hipSetDevice(c->device));
  c->cancel.store(0);
  // order after the caller's queued work
  if (!c->fork_ev) {
    HIP_TRY(c, hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming));
    HIP_TRY(c, hipEventCreateWithFlags(&c->join_ev, hipEventDisableTiming));
  }
  HIP_TRY(c, hipEventRecord(c->fork_ev, c->stream));
  HIP_TRY(c, hipStreamWaitEvent(b->stream, c->fork_ev, 0));
  const size_t n = b->plans.size();
  if (b->graphed) {
    // the captured contractions write the caller's device outputs directly
    std::vector<double *> want(n);
    for (size_t i = 0; i < n; ++i) want[i] = outs_on_device && b->job_out[i] ? outs[i] : b->res[i];
    if (want != b->cur_tab) {
      HIP_TRY(c, hipStreamSynchronize(b->stream));  // the previous copy may still read the pinned table
      for (size_t i = 0; i < n; ++i) b->h_out_tab[i] = want[i];
      HIP_TRY(c, hipMemcpyAsync(b->d_out_tab, b->h_out_tab, n * sizeof(double *), hipMemcpyHostToDevice, b->stream));
      b->cur_tab = want;
    }
    HIP_TRY(c, hipGraphLaunch(b->exec, b->stream));
  } else {
    BatchScope scope(b, true);
    c->replay_uploads = true;
    ccut_status st = batch_enqueue(b, false);
    if (st != CCUT_OK) return st;
  }
  if (!outs_on_device) {
    for (size_t i = 0; i < n; ++i)
      HIP_TRY(c, hipMemcpyAsync(outs[i], b->res[i], sizeof(double) << b->qubits[i].size(), hipMemcpyDeviceToHost,
                                b->stream));
    HIP_TRY(c, hipStreamSynchronize(b->stream));
    return CCUT_OK;
  }
  // device outputs not written in place (an eager run, or a plan whose
  // contraction has a launch of its own): one gather launch; then the
  // caller's stream waits for the batch (no host synchronization)
  if (n == 0) return CCUT_OK;
  if (!b->d_copy) {
    HIP_TRY(c, hipHostMalloc((void **)&b->h_copy, n * sizeof(OutCopy), hipHostMallocDefault));
    HIP_TRY(c, hipMalloc((void **)&b->d_copy, n * sizeof(OutCopy)));
    HIP_TRY(c, hipEventCreateWithFlags(&b->done_ev, hipEventDisableTiming));
  }
  std::vector<double *> key(outs, outs + n);
  key.push_back(b->graphed ? (double *)1 : nullptr);  // the copy list depends on the mode too
  size_t n_copy = 0;
  uint64_t max_n = 0;
  for (size_t i = 0; i < n; ++i)
    if (!b->graphed || !b->job_out[i]) {
      ++n_copy;
      max_n = std::max<uint64_t>(max_n, uint64_t(1) << b->qubits[i].size());
    }
  if (key != b->last_outs) {
    // the previous run's gather may still read both copies of the list
    HIP_TRY(c, hipStreamSynchronize(b->stream));
    size_t k = 0;
    for (size_t i = 0; i < n; ++i)
      if (!b->graphed || !b->job_out[i]) b->h_copy[k++] = OutCopy{b->res[i], outs[i], uint64_t(1) << b->qubits[i].size()};
    if (n_copy)
      HIP_TRY(c, hipMemcpyAsync(b->d_copy, b->h_copy, n_copy * sizeof(OutCopy), hipMemcpyHostToDevice, b->stream));
    b->last_outs = key;
  }
  for (size_t i0 = 0; i0 < n_copy; i0 += 65535)
    HIP_TRY(c, launch_gather_f64(b->d_copy + i0, (uint32_t)std::min<size_t>(65535, n_copy - i0), max_n, b->stream));
  HIP_TRY(c, hipEventRecord(b->done_ev, b->stream));
  HIP_TRY(c, hipStreamWaitEvent(c->stream, b->done_ev, 0));
  return CCUT_OK;
}

ccut_status ccut_batch_info(const ccut_batch *b, uint64_t *n_items, uint32_t *block, uint32_t *grid,
                            int32_t *tune_cached, int32_t *graphed, double *models_ms) {
  if (!b) return CCUT_E_INVALID;
  if (n_items) *n_items = b->items.size();
  if (block) *block = b->block;
  if (grid) *grid = b->grid;
  if (tune_cached) *tune_cached = (int32_t)b->tune_cached;
  if (graphed) *graphed = b->graphed ? 1 : 0;
  if (models_ms) *models_ms = b->tuned_ms;
  return CCUT_OK;
}

void ccut_batch_destroy(ccut_batch *b) {
  if (!b) return;
  ccut_ctx *c = b->ctx;
  if (c && c->device >= 0) {
    (void)hipSetDevice(c->device);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
  }
  delete b;
  ctx_release(c);
}

ccut_status ccut_run_batch(ccut_ctx *c, ccut_plan *const *plans, size_t n, const ccut_eval_opts *eo,
                           const uint32_t *const *qubits, const uint32_t *nq, double *const *outs) {
  ccut_batch *b = nullptr;
  ccut_status st = ccut_batch_create(c, plans, n, eo, qubits, nq, 0, &b);
  if (st != CCUT_OK) return st;
  st = ccut_batch_run(b, outs, 0);
  ccut_batch_destroy(b);
  return st;
}

}  // extern "C"

// ================================================= learned term proposal

struct ccut_mlp {
  ccut_ctx *ctx = nullptr;
  uint32_t F = 0, H = 0;
  uint64_t n_params = 0;
  uint64_t off_w1 = 0, off_b1 = 0, off_w2 = 0, off_b2 = 0, off_w3 = 0, off_b3 = 0, off_w4 = 0, off_b4 = 0;
  Arena arena;  // parameters and Adam state
  Arena work;   // activations, regrown when a call needs more rows
  uint64_t work_rows = 0;
  float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  uint16_t *pb = nullptr;  // bf16 copy of the parameters used by the products
  uint64_t t = 0;          // Adam step count
  uint16_t *xb = nullptr, *h1 = nullptr, *h2 = nullptr, *h3 = nullptr, *d1 = nullptr, *d2 = nullptr, *d3 = nullptr;
  float *y = nullptr, *tb = nullptr, *dy = nullptr, *sq = nullptr, *part = nullptr;
  ~ccut_mlp() {
    if (ctx && ctx->device >= 0) {
      (void)hipSetDevice(ctx->device);
      (void)hipStreamSynchronize(ctx->stream);
    }
    arena.release();
    work.release();
  }
};

struct ccut_learned {
  ccut_ctx *ctx = nullptr;
  ccut_plan *plan = nullptr;
  uint32_t k = 0, nq = 0, width = 64, circuit = 0;
  int32_t precision = CCUT_FP64;  // of the exhaustive contraction
  uint64_t K = 0;
  Arena arena;  // fragment tensors, norms, share tables
  std::vector<std::vector<char>> staged;
  RecombArgs args{};
  LearnedDev h{};
  LearnedDev *d = nullptr;
  ~ccut_learned() {
    if (ctx && ctx->device >= 0) {
      (void)hipSetDevice(ctx->device);
      (void)hipStreamSynchronize(ctx->stream);
    }
    arena.release();
  }
};

namespace {

// Run with the context's allocations going to another arena (long-lived
// objects), everything on the context stream.
struct ArenaScope {
  ccut_ctx *c;
  Arena *a;
  std::vector<std::vector<char>> *st;
  bool saved_aux;
  ArenaScope(ccut_ctx *cc, Arena *aa, std::vector<std::vector<char>> *ss) : c(cc), a(aa), st(ss) {
    std::swap(c->arena, *a);
    std::swap(c->staged, *st);
    saved_aux = c->use_aux;
    c->use_aux = false;
    c->cur = c->stream;
  }
  ~ArenaScope() {
    std::swap(c->arena, *a);
    std::swap(c->staged, *st);
    c->use_aux = saved_aux;
  }
};

ccut_status begin_call(ccut_ctx *c) {
  if (!c) return CCUT_E_INVALID;
  if (c->device < 0) return fail(c, CCUT_E_DEVICE, "host-only context: evaluation needs a device");
  HIP_TRY(c, hipSetDevice(c->device));
  c->cancel.store(0);
  c->arena.reset();
  c->staged.clear();
  c->cur = c->stream;
  HIP_TRY(c, pin_begin(c));
  return CCUT_OK;
}

ccut_status sync_call(ccut_ctx *c) {
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return CCUT_OK;
}

ccut_status mlp_gemm(ccut_ctx *c, const uint16_t *A, uint64_t sam, uint64_t sak, const uint16_t *B, uint64_t sbk,
                     uint64_t sbn, uint64_t M, uint32_t N, uint32_t K, void *C, uint64_t ldc, int epi,
                     const float *bias = nullptr, const uint16_t *mask = nullptr, uint64_t ldm = 0) {
  MlpGemm g{A, sam, sak, B, sbk, sbn, M, N, K, C, ldc, bias, mask, ldm};
  HIP_TRY(c, launch_mlp_gemm(g, epi, c->cur));
  return CCUT_OK;
}

ccut_status mlp_ensure_work(ccut_mlp *M, uint64_t rows) {
  ccut_ctx *c = M->ctx;
  if (rows <= M->work_rows) return CCUT_OK;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  M->work.release();
  const uint64_t F = M->F, H = M->H;
  auto b16 = [&](uint64_t n) { return (uint16_t *)M->work.get(n * 2); };
  auto f32 = [&](uint64_t n) { return (float *)M->work.get(n * 4); };
  M->xb = b16(rows * F);
  M->h1 = b16(rows * H);
  M->h2 = b16(rows * H);
  M->h3 = b16(rows * H);
  M->d1 = b16(rows * H);
  M->d2 = b16(rows * H);
  M->d3 = b16(rows * H);
  M->y = f32(rows);
  M->tb = f32(rows);
  M->dy = f32(rows);
  M->sq = f32(rows);
  M->part = f32((uint64_t)colsum_chunks(rows) * std::max(H, F));
  if (!M->xb || !M->h1 || !M->h2 || !M->h3 || !M->d1 || !M->d2 || !M->d3 || !M->y || !M->tb || !M->dy || !M->sq ||
      !M->part) {
    M->work.release();
    M->work_rows = 0;
    return fail(c, CCUT_E_OOM, "device allocation failed");
  }
  M->work_rows = rows;
  return CCUT_OK;
}

// h1..h3 and y for rows of x (rows <= work_rows)
ccut_status mlp_forward_rows(ccut_mlp *M, const uint16_t *x, uint64_t rows, float *y, float scale = 1.f) {
  ccut_ctx *c = M->ctx;
  const uint32_t F = M->F, H = M->H;
  ccut_status st;
  KTimer t(c, CCUT_K_MLP);
  if ((st = mlp_gemm(c, x, F, 1, M->pb + M->off_w1, 1, F, rows, H, F, M->h1, H, MLP_EPI_BIAS_RELU,
                     M->p + M->off_b1)) != CCUT_OK)
    return st;
  if ((st = mlp_gemm(c, M->h1, H, 1, M->pb + M->off_w2, 1, H, rows, H, H, M->h2, H, MLP_EPI_BIAS_RELU,
                     M->p + M->off_b2)) != CCUT_OK)
    return st;
  if ((st = mlp_gemm(c, M->h2, H, 1, M->pb + M->off_w3, 1, H, rows, H, H, M->h3, H, MLP_EPI_BIAS_RELU,
                     M->p + M->off_b3)) != CCUT_OK)
    return st;
  HIP_TRY(c, launch_head_forward(M->h3, H, rows, M->pb + M->off_w4, M->p + M->off_b4, scale, y, c->cur));
  return CCUT_OK;
}

// Gradient of the mean squared error into M->g after mlp_forward_rows on
// the same rows; loss_sum (device) receives sum (y - t)^2.
ccut_status mlp_backward_rows(ccut_mlp *M, const uint16_t *x, const float *t, uint64_t rows, float *loss_sum) {
  ccut_ctx *c = M->ctx;
  const uint32_t F = M->F, H = M->H;
  const uint32_t R = (uint32_t)rows;
  ccut_status st;
  KTimer tm(c, CCUT_K_MLP);
  HIP_TRY(c, launch_head_backward(M->h3, H, rows, M->pb + M->off_w4, M->y, t, M->dy, M->sq, M->d3, c->cur));
  HIP_TRY(c, launch_colsum(M->h3, H, rows, M->dy, M->part, M->g + M->off_w4, c->cur));
  HIP_TRY(c, launch_vsum(M->dy, rows, M->g + M->off_b4, c->cur));
  HIP_TRY(c, launch_vsum(M->sq, rows, loss_sum, c->cur));
  // layer 3: dW3 = dZ3^T H2, db3 = colsum dZ3, dZ2 = (dZ3 W3) [H2 > 0]
  const uint16_t *hin[3] = {x, M->h1, M->h2};
  uint16_t *dz[3] = {M->d1, M->d2, M->d3};
  const uint64_t offw[3] = {M->off_w1, M->off_w2, M->off_w3}, offb[3] = {M->off_b1, M->off_b2, M->off_b3};
  for (int l = 2; l >= 0; --l) {
    const uint32_t in = l == 0 ? F : H;
    if ((st = mlp_gemm(c, dz[l], 1, H, hin[l], in, 1, H, in, R, M->g + offw[l], in, MLP_EPI_F32)) != CCUT_OK)
      return st;
    HIP_TRY(c, launch_colsum(dz[l], H, rows, nullptr, M->part, M->g + offb[l], c->cur));
    if (l > 0 && (st = mlp_gemm(c, dz[l], H, 1, M->pb + offw[l], H, 1, rows, H, H, dz[l - 1], H, MLP_EPI_MASK,
                                nullptr, hin[l], H)) != CCUT_OK)
      return st;
  }
  return CCUT_OK;
}

uint64_t splitmix64(uint64_t &s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace

extern "C" {

ccut_status ccut_mlp_create(ccut_ctx *c, uint32_t F, uint32_t H, ccut_mlp **out) {
  if (!out) return fail(c, CCUT_E_INVALID, "out is NULL");
  *out = nullptr;
  ccut_status st = begin_call(c);
  if (st != CCUT_OK) return st;
  if (F == 0 || H == 0 || F % 64 || H % 64 || F > 256 || H > 256)
    return fail(c, CCUT_E_INVALID, "F and H must be multiples of 64 in [64, 256]");
  std::unique_ptr<ccut_mlp> M(new (std::nothrow) ccut_mlp());
  if (!M) return fail(c, CCUT_E_OOM, "host allocation failed");
  M->ctx = c;
  M->F = F;
  M->H = H;
  M->arena.alloc = M->work.alloc = c->arena.alloc;
  M->arena.free_fn = M->work.free_fn = c->arena.free_fn;
  M->arena.user = M->work.user = c->arena.user;
  uint64_t o = 0;
  M->off_w1 = o;
  o += (uint64_t)H * F;
  M->off_b1 = o;
  o += H;
  M->off_w2 = o;
  o += (uint64_t)H * H;
  M->off_b2 = o;
  o += H;
  M->off_w3 = o;
  o += (uint64_t)H * H;
  M->off_b3 = o;
  o += H;
  M->off_w4 = o;
  o += H;
  M->off_b4 = o;
  o += 1;
  M->n_params = o;
  M->p = (float *)M->arena.get(o * 4);
  M->g = (float *)M->arena.get(o * 4);
  M->m = (float *)M->arena.get(o * 4);
  M->v = (float *)M->arena.get(o * 4);
  M->pb = (uint16_t *)M->arena.get(o * 2);
  if (!M->p || !M->g || !M->m || !M->v || !M->pb) return fail(c, CCUT_E_OOM, "device allocation failed");
  // He-style uniform initialisation (limits sqrt(6 / fan_in), output layer
  // sqrt(3 / fan_in)), biases zero
  std::vector<float> init(o, 0.f);
  uint64_t s = 0x5EED0000A11CE5ull;
  auto fill = [&](uint64_t off, uint64_t count, double lim) {
    for (uint64_t i = 0; i < count; ++i) {
      const double u = (double)(splitmix64(s) >> 11) * (1.0 / 9007199254740992.0);
      init[off + i] = (float)((2.0 * u - 1.0) * lim);
    }
  };
  fill(M->off_w1, (uint64_t)H * F, std::sqrt(6.0 / F));
  fill(M->off_w2, (uint64_t)H * H, std::sqrt(6.0 / H));
  fill(M->off_w3, (uint64_t)H * H, std::sqrt(6.0 / H));
  fill(M->off_w4, H, std::sqrt(3.0 / H));
  ccut_mlp *raw = M.get();
  st = ccut_mlp_set_params(raw, init.data(), init.size());
  if (st != CCUT_OK) return st;
  *out = M.release();
  ctx_retain(c);
  return CCUT_OK;
}

ccut_status ccut_mlp_set_params(ccut_mlp *M, const float *params, size_t count) {
  if (!M || !params) return CCUT_E_INVALID;
  ccut_ctx *c = M->ctx;
  ccut_status st = begin_call(c);
  if (st != CCUT_OK) return st;
  if (count != M->n_params) return fail(c, CCUT_E_INVALID, "parameter count does not match the network");
  HIP_TRY(c, hipMemcpyAsync(M->p, params, count * 4, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemsetAsync(M->m, 0, count * 4, c->stream));
  HIP_TRY(c, hipMemsetAsync(M->v, 0, count * 4, c->stream));
  HIP_TRY(c, launch_to_bf16(M->p, M->pb, count, c->stream));
  M->t = 0;
  return sync_call(c);
}

ccut_status ccut_mlp_get_params(ccut_mlp *M, float *params, size_t count) {
  if (!M || !params) return CCUT_E_INVALID;
  ccut_ctx *c = M->ctx;
  ccut_status st = begin_call(c);
  if (st != CCUT_OK) return st;
  if (count != M->n_params) return fail(c, CCUT_E_INVALID, "parameter count does not match the network");
  HIP_TRY(c, hipMemcpyAsync(params, M->p, count * 4, hipMemcpyDeviceToHost, c->stream));
  return sync_call(c);
}

ccut_status ccut_mlp_forward(ccut_mlp *M, const uint16_t *x, uint64_t n, float *y) {
  if (!M) return CCUT_E_INVALID;
  ccut_ctx *c = M->ctx;
  ccut_status st = begin_call(c);
  if (st != CCUT_OK) return st;
  if (n && (!x || !y)) return fail(c, CCUT_E_INVALID, "NULL argument");
  const uint64_t chunk = std::min<uint64_t>(n, 1ull << 18);
  if ((st = mlp_ensure_work(M, std::max<uint64_t>(chunk, 64))) != CCUT_OK) return st;
  for (uint64_t r0 = 0; r0 < n; r0 += chunk)
    if ((st = mlp_forward_rows(M, x + r0 * M->F, std::min(chunk, n - r0), y + r0)) != CCUT_OK) return st;
  return sync_call(c);
}

ccut_status ccut_mlp_gradients(ccut_mlp *M, const uint16_t *x, const float *t, uint64_t n, float *grads,
                               double *loss) {
  if (!M) return CCUT_E_INVALID;
  ccut_ctx *c = M->ctx;
  ccut_status st = begin_call(c);
  if (st != CCUT_OK) return st;
  if (!x || !t || !grads) return fail(c, CCUT_E_INVALID, "NULL argument");
  if (n == 0 || n % 64 || n > (1ull << 24)) return fail(c, CCUT_E_INVALID, "n must be a positive multiple of 64");
  if ((st = mlp_ensure_work(M, n)) != CCUT_OK) return st;
  float *lsum = aget<float>(c, 1);
  if (!lsum) return fail(c, CCUT_E_OOM, "device allocation failed");
  if ((st = mlp_forward_rows(M, x, n, M->y)) != CCUT_OK) return st;
  if ((st = mlp_backward_rows(M, x, t, n, lsum)) != CCUT_OK) return st;
  float hl = 0.f;
  HIP_TRY(c, hipMemcpyAsync(grads, M->g, M->n_params * 4, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(&hl, lsum, 4, hipMemcpyDeviceToHost, c->stream));
  if ((st = sync_call(c)) != CCUT_OK) return st;
  if (loss) *loss = (double)hl / (double)n;
  return CCUT_OK;
}

ccut_status ccut_mlp_train(ccut_mlp *M, const uint16_t *x, const float *t, uint64_t n, uint32_t batch,
                           uint32_t steps, float lr, uint64_t seed, float *losses) {
  if (!M) return CCUT_E_INVALID;
  ccut_ctx *c = M->ctx;
  ccut_status st = begin_call(c);
  if (st != CCUT_OK) return st;
  if (!x || !t) return fail(c, CCUT_E_INVALID, "NULL argument");
  if (n == 0 || batch == 0 || batch % 64 || batch > n || batch > (1u << 24))
    return fail(c, CCUT_E_INVALID, "batch must be a positive multiple of 64, at most n");
  if ((st = mlp_ensure_work(M, batch)) != CCUT_OK) return st;
  float *lsum = aget<float>(c, std::max<uint32_t>(steps, 1));
  if (!lsum) return fail(c, CCUT_E_OOM, "device allocation failed");
  const int in_order = batch == n;
  for (uint32_t s = 0; s < steps; ++s) {
    HIP_TRY(c, launch_gather_rows(x, t, n, M->F, batch, s, seed, in_order, M->xb, M->tb, c->stream));
    if ((st = mlp_forward_rows(M, M->xb, batch, M->y)) != CCUT_OK) return st;
    if ((st = mlp_backward_rows(M, M->xb, M->tb, batch, lsum + s)) != CCUT_OK) return st;
    M->t += 1;
    const float c1 = (float)(1.0 - std::pow(0.9, (double)M->t));
    const float c2 = (float)(1.0 - std::pow(0.999, (double)M->t));
    KTimer tm(c, CCUT_K_MLP);
    HIP_TRY(c, launch_adam(M->p, M->g, M->m, M->v, M->pb, M->n_params, lr, 0.9f, 0.999f, c1, c2, 1e-8f, c->stream));
  }
  if (losses && steps) {
    HIP_TRY(c, hipMemcpyAsync(losses, lsum, steps * 4, hipMemcpyDeviceToHost, c->stream));
    if ((st = sync_call(c)) != CCUT_OK) return st;
    for (uint32_t s = 0; s < steps; ++s) losses[s] /= (float)batch;
    return CCUT_OK;
  }
  return sync_call(c);
}

void ccut_mlp_destroy(ccut_mlp *M) {
  if (!M) return;
  ccut_ctx *c = M->ctx;
  delete M;
  ctx_release(c);
}

ccut_status ccut_learned_create(ccut_plan *p, const ccut_eval_opts *eo, const uint32_t *qubits, uint32_t nq,
                                ccut_learned **out) {
  if (!p || !out) return CCUT_E_INVALID;
  *out = nullptr;
  ccut_status st = check_eval(p, eo);
  if (st != CCUT_OK) return st;
  ccut_ctx *c = p->ctx;
  if ((st = check_request(c, p->pd.n, qubits, nq)) != CCUT_OK) return st;
  const PlanData &pd = p->pd;
  if (pd.frags.size() > (size_t)kMaxFrags) return fail(c, CCUT_E_UNSUPPORTED, "more than 64 fragments");
  if (pd.k == 0 || pd.k > 12) return fail(c, CCUT_E_UNSUPPORTED, "the term model needs 1 to 12 cuts");
  if (eo->flags & CCUT_FLAG_ML) return fail(c, CCUT_E_UNSUPPORTED, "the maximum-likelihood correction applies to marginals");
  std::unique_ptr<ccut_learned> L(new (std::nothrow) ccut_learned());
  if (!L) return fail(c, CCUT_E_OOM, "host allocation failed");
  L->ctx = c;
  L->plan = p;
  L->k = pd.k;
  L->K = 1ull << (2 * pd.k);
  L->nq = nq;
  L->circuit = eo->circuit;
  L->precision = eo->precision;
  L->width = (uint32_t)((6 * pd.k + 63) / 64 * 64);
  L->arena.alloc = c->arena.alloc;
  L->arena.free_fn = c->arena.free_fn;
  L->arena.user = c->arena.user;
  {
    ArenaScope scope(c, &L->arena, &L->staged);
    RecombArgs &args = L->args;
    args.n_frags = (uint32_t)pd.frags.size();
    args.k = pd.k;
    uint64_t n_slots = 0;
    std::vector<uint64_t> slot_off(pd.frags.size());
    for (const Fragment &f : pd.frags) {
      slot_off[f.index] = n_slots;
      n_slots += 4 * f.axes.size();
    }
    double *shares = aget<double>(c, std::max<uint64_t>(n_slots, 1));
    if (!shares) return fail(c, CCUT_E_OOM, "device allocation failed");
    std::vector<int64_t> src(2 * pd.k, -1);
    LearnedDev &h = L->h;
    h.k = pd.k;
    h.n_frags = args.n_frags;
    for (const Fragment &f : pd.frags) {
      FragRequest r = marginal_request(f, qubits, nq);
      double *dist = nullptr, *T = nullptr;
      if (use_heisenberg(f, eo, r.req_pos.size())) {
        if ((st = heis_tensor(p, f, r, eo->circuit, nullptr, &T)) != CCUT_OK) return st;
      } else {
        if ((st = variant_dists(p, eo, f, r, &dist)) != CCUT_OK) return st;
        if ((st = pauli_passes(c, f, r, dist, 1ull << r.meas.size(), 0, &T)) != CCUT_OK) return st;
      }
      RecombFrag &rf = args.f[f.index];
      rf.T = T;
      rf.n_axes = (uint32_t)f.axes.size();
      rf.rows = 1u << r.req_pos.size();
      rf.n_req = (uint32_t)r.req_pos.size();
      for (size_t j = 0; j < f.axes.size(); ++j) rf.axis_cut[j] = f.axes[j].cut;
      for (size_t i = 0; i < r.req_user.size(); ++i) rf.req_user[i] = r.req_user[i];
      const uint32_t a = (uint32_t)f.axes.size();
      const uint64_t ncols = 1ull << (2 * a);
      double *norm = aget<double>(c, ncols);
      double *part = aget<double>(c, (uint64_t)4 * std::max<uint32_t>(a, 1) * share_chunks(a));
      if (!norm || !part) return fail(c, CCUT_E_OOM, "device allocation failed");
      {
        KTimer t(c, CCUT_K_TERMS);
        HIP_TRY(c, launch_colnorm(T, rf.rows, ncols, norm, c->cur));
        HIP_TRY(c, launch_shares(norm, a, part, shares + slot_off[f.index], c->cur));
      }
      h.norm[f.index] = norm;
      h.n_axes[f.index] = a;
      for (uint32_t j = 0; j < a; ++j) {
        h.axis_cut[f.index][j] = f.axes[j].cut;
        src[2 * f.axes[j].cut + f.axes[j].side] = (int64_t)(slot_off[f.index] + 4 * j);
      }
    }
    int64_t *d_src = (int64_t *)upload(c, src.data(), src.size() * 8);
    double *phi = aget<double>(c, 8 * pd.k);
    if (!d_src || !phi) return fail(c, CCUT_E_OOM, "device allocation failed");
    HIP_TRY(c, launch_phi(shares, d_src, pd.k, phi, c->cur));
    h.phi = phi;
    L->d = (LearnedDev *)upload(c, &h, sizeof(h));
    if (!L->d) return fail(c, CCUT_E_OOM, "device allocation failed");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  *out = L.release();
  ctx_retain(c);
  return CCUT_OK;
}

ccut_status ccut_learned_info(const ccut_learned *L, uint32_t *k, uint64_t *n_terms, uint32_t *width) {
  if (!L) return CCUT_E_INVALID;
  if (k) *k = L->k;
  if (n_terms) *n_terms = L->K;
  if (width) *width = L->width;
  return CCUT_OK;
}

ccut_status ccut_learned_features(ccut_learned *L, const uint64_t *terms, uint64_t first, uint64_t n, uint16_t *x) {
  if (!L) return CCUT_E_INVALID;
  ccut_ctx *c = L->ctx;
  ccut_status st = begin_call(c);
  if (st != CCUT_OK) return st;
  if (n && !x) return fail(c, CCUT_E_INVALID, "x is NULL");
  if (!terms && (first > L->K || n > L->K - first)) return fail(c, CCUT_E_INVALID, "term range beyond 4^k");
  {
    KTimer t(c, CCUT_K_TERMS);
    HIP_TRY(c, launch_features(L->d, terms, first, n, L->width, x, c->cur));
  }
  return sync_call(c);
}

ccut_status ccut_learned_log_weights(ccut_learned *L, const uint64_t *terms, uint64_t first, uint64_t n, int kind,
                                     float *y) {
  if (!L) return CCUT_E_INVALID;
  ccut_ctx *c = L->ctx;
  ccut_status st = begin_call(c);
  if (st != CCUT_OK) return st;
  if (n && !y) return fail(c, CCUT_E_INVALID, "y is NULL");
  if (kind < 0 || kind > 2) return fail(c, CCUT_E_INVALID, "kind must be 0, 1 or 2");
  if (!terms && (first > L->K || n > L->K - first)) return fail(c, CCUT_E_INVALID, "term range beyond 4^k");
  {
    KTimer t(c, CCUT_K_TERMS);
    HIP_TRY(c, launch_labels(L->d, terms, first, n, y, kind, c->cur));
  }
  return sync_call(c);
}

ccut_status ccut_learned_support(ccut_learned *L, uint64_t cap, uint64_t *terms, uint64_t *count) {
  if (!L || !count) return CCUT_E_INVALID;
  ccut_ctx *c = L->ctx;
  ccut_status st = begin_call(c);
  if (st != CCUT_OK) return st;
  if (cap && !terms) return fail(c, CCUT_E_INVALID, "terms is NULL");
  uint64_t *flags = aget<uint64_t>(c, L->K), *pos = aget<uint64_t>(c, L->K);
  uint64_t *scratch = aget<uint64_t>(c, scan_scratch_words(L->K));
  if (!flags || !pos || !scratch) return fail(c, CCUT_E_OOM, "device allocation failed");
  {
    KTimer t(c, CCUT_K_TERMS);
    HIP_TRY(c, launch_support(L->d, L->K, flags, pos, scratch, cap, terms, c->cur));
  }
  HIP_TRY(c, hipMemcpyAsync(count, pos + L->K - 1, 8, hipMemcpyDeviceToHost, c->stream));
  return sync_call(c);
}

}  // extern "C"

namespace {
// The network's logits over every term of L, enqueued on the context's
// stream (no synchronization).
ccut_status learned_logits_enqueue(ccut_learned *L, ccut_mlp *M, float *logits) {
  ccut_ctx *c = L->ctx;
  ccut_status st;
  if (!logits) return fail(c, CCUT_E_INVALID, "logits is NULL");
  if (M->ctx != c || M->F != L->width) return fail(c, CCUT_E_INVALID, "network input width differs from the features");
  if (M->F == 64 && M->H == 256) {  // the whole pass in one launch, activations on chip
    MlpFused net{};
    net.w1 = M->pb + M->off_w1;
    net.w2 = M->pb + M->off_w2;
    net.w3 = M->pb + M->off_w3;
    net.w4 = M->pb + M->off_w4;
    net.b1 = M->p + M->off_b1;
    net.b2 = M->p + M->off_b2;
    net.b3 = M->p + M->off_b3;
    net.b4 = M->p + M->off_b4;
    net.F = M->F;
    net.H = M->H;
    {
      KTimer t(c, CCUT_K_MLP);
      HIP_TRY(c, launch_mlp_logits_fused(L->d, net, 0, L->K, kLabelScale, logits, c->cur));
    }
    return CCUT_OK;
  }
  const uint64_t chunk = std::min<uint64_t>(L->K, 1ull << 18);
  if ((st = mlp_ensure_work(M, std::max<uint64_t>(chunk, 64))) != CCUT_OK) return st;
  uint16_t *x = aget<uint16_t>(c, chunk * L->width);
  if (!x) return fail(c, CCUT_E_OOM, "device allocation failed");
  for (uint64_t first = 0; first < L->K; first += chunk) {
    const uint64_t rows = std::min(chunk, L->K - first);
    {
      KTimer t(c, CCUT_K_TERMS);
      HIP_TRY(c, launch_features(L->d, nullptr, first, rows, L->width, x, c->cur));
    }
    if ((st = mlp_forward_rows(M, x, rows, logits + first, kLabelScale)) != CCUT_OK) return st;
  }
  return CCUT_OK;
}

}  // namespace

extern "C" {

ccut_status ccut_learned_logits(ccut_learned *L, ccut_mlp *M, float *logits) {
  if (!L || !M) return CCUT_E_INVALID;
  ccut_ctx *c = L->ctx;
  ccut_status st = begin_call(c);
  if (st != CCUT_OK) return st;
  if ((st = learned_logits_enqueue(L, M, logits)) != CCUT_OK) return st;
  return sync_call(c);
}

ccut_status ccut_proposal(ccut_ctx *c, const float *logits, uint64_t K, double eps, double *q) {
  ccut_status st = begin_call(c);
  if (st != CCUT_OK) return st;
  if (!q || K == 0) return fail(c, CCUT_E_INVALID, "q is NULL or K is 0");
  if (!(eps >= 0.0 && eps <= 1.0)) return fail(c, CCUT_E_INVALID, "eps must be in [0, 1]");
  const uint32_t nb = reduce_blocks(K);
  float *mpart = aget<float>(c, nb);
  double *spart = aget<double>(c, nb), *stats = aget<double>(c, 2);
  if (!mpart || !spart || !stats) return fail(c, CCUT_E_OOM, "device allocation failed");
  {
    KTimer t(c, CCUT_K_TERMS);
    HIP_TRY(c, launch_proposal(logits, K, eps, mpart, spart, stats, q, c->cur));
  }
  return sync_call(c);
}

}  // extern "C"

namespace {
ccut_status draw_terms(ccut_ctx *c, const double *q, uint64_t K, uint64_t n, uint64_t seed, uint64_t cid,
                       uint64_t *out) {
  uint64_t *cdf = aget<uint64_t>(c, K), *scratch = aget<uint64_t>(c, scan_scratch_words(K));
  if (!cdf || !scratch) return fail(c, CCUT_E_OOM, "device allocation failed");
  KTimer t(c, CCUT_K_TERMS);
  HIP_TRY(c, launch_int_cdf(q, K, cdf, scratch, c->cur));
  HIP_TRY(c, launch_sample_terms(cdf, K, n, seed, cid, out, c->cur));
  return CCUT_OK;
}
}  // namespace

extern "C" {

ccut_status ccut_sample_terms(ccut_ctx *c, const double *q, uint64_t K, uint64_t n, uint64_t seed, uint64_t cid,
                              uint64_t *out) {
  ccut_status st = begin_call(c);
  if (st != CCUT_OK) return st;
  if (!q || K == 0 || (n && !out)) return fail(c, CCUT_E_INVALID, "NULL argument or K = 0");
  if (n > 0xFFFFFFFFull) return fail(c, CCUT_E_INVALID, "at most 2^32 - 1 terms per draw");
  if ((st = draw_terms(c, q, K, n, seed, cid, out)) != CCUT_OK) return st;
  return sync_call(c);
}

ccut_status ccut_learned_estimate(ccut_learned *L, const double *q, uint64_t n, uint64_t seed, double *out,
                                  int on_device, uint64_t *terms_out) {
  if (!L) return CCUT_E_INVALID;
  ccut_ctx *c = L->ctx;
  ccut_status st = begin_call(c);
  if (st != CCUT_OK) return st;
  if (!q || !out) return fail(c, CCUT_E_INVALID, "NULL argument");
  if (n == 0 || n > 0xFFFFFFFFull) return fail(c, CCUT_E_INVALID, "n must be in [1, 2^32)");
  uint64_t *terms = terms_out ? terms_out : aget<uint64_t>(c, n);
  double *scale = aget<double>(c, n), *res = aget<double>(c, (size_t)1 << L->nq);
  if (!terms || !scale || !res) return fail(c, CCUT_E_OOM, "device allocation failed");
  if ((st = draw_terms(c, q, L->K, n, seed, L->circuit, terms)) != CCUT_OK) return st;
  {
    KTimer t(c, CCUT_K_TERMS);
    HIP_TRY(c, launch_is_scale(terms, q, n, scale, c->cur));
  }
  GemmArgs g;
  make_gemm_args(L->args, g);
  g.terms = terms;
  g.tscale = scale;
  g.K = n;
  if ((st = run_gemm(c, g, false, res)) != CCUT_OK) return st;
  return finish_out(c, res, out, (size_t)1 << L->nq, on_device);
}

ccut_status ccut_learned_exhaustive(ccut_learned *L, double *out, int on_device) {
  if (!L) return CCUT_E_INVALID;
  ccut_ctx *c = L->ctx;
  ccut_status st = begin_call(c);
  if (st != CCUT_OK) return st;
  if (!out) return fail(c, CCUT_E_INVALID, "out is NULL");
  double *res = aget<double>(c, (size_t)1 << L->nq);
  if (!res) return fail(c, CCUT_E_OOM, "device allocation failed");
  RecombArgs args = L->args;
  args.lo_parts = L->precision == CCUT_FP32X3_MFMA_FP64SUM;
  if ((st = recombine(c, args, L->nq, L->precision != CCUT_FP64, res)) != CCUT_OK) return st;
  return finish_out(c, res, out, (size_t)1 << L->nq, on_device);
}

void ccut_learned_destroy(ccut_learned *L) {
  if (!L) return;
  ccut_ctx *c = L->ctx;
  delete L;
  ctx_release(c);
}

ccut_status ccut_learned_marginal(ccut_plan *p, const ccut_eval_opts *eo, ccut_mlp *net, uint64_t n_terms,
                                  const uint32_t *qubits, uint32_t nq, double *out, int out_on_device,
                                  double *out_stderr_l1) {
  if (!p || !eo || !net) return CCUT_E_INVALID;
  ccut_ctx *c = p->ctx;
  if (!out) return fail(c, CCUT_E_INVALID, "out is NULL");
  if (n_terms == 0 || n_terms > 0xFFFFFFFFull) return fail(c, CCUT_E_INVALID, "n_terms must be in [1, 2^32)");
  ccut_learned *L = nullptr;
  ccut_status st = ccut_learned_create(p, eo, qubits, nq, &L);
  if (st != CCUT_OK) return st;
  std::unique_ptr<ccut_learned, void (*)(ccut_learned *)> hold(L, ccut_learned_destroy);
  if ((st = begin_call(c)) != CCUT_OK) return st;
  const uint64_t K = L->K, bins = 1ull << L->nq;
  const uint32_t nb = reduce_blocks(K);
  float *logits = aget<float>(c, K), *mpart = aget<float>(c, nb);
  double *q = aget<double>(c, K), *spart = aget<double>(c, nb), *stats = aget<double>(c, 2);
  uint64_t *terms = aget<uint64_t>(c, n_terms);
  double *scale = aget<double>(c, n_terms), *res = aget<double>(c, bins);
  double *res2 = out_stderr_l1 ? aget<double>(c, bins) : nullptr;
  if (!logits || !mpart || !q || !spart || !stats || !terms || !scale || !res || (out_stderr_l1 && !res2))
    return fail(c, CCUT_E_OOM, "device allocation failed");
  if ((st = learned_logits_enqueue(L, net, logits)) != CCUT_OK) return st;
  {
    KTimer t(c, CCUT_K_TERMS);
    HIP_TRY(c, launch_proposal(logits, K, 0.05, mpart, spart, stats, q, c->cur));
  }
  if ((st = draw_terms(c, q, K, n_terms, eo->seed, L->circuit, terms)) != CCUT_OK) return st;
  {
    KTimer t(c, CCUT_K_TERMS);
    HIP_TRY(c, launch_is_scale(terms, q, n_terms, scale, c->cur));
  }
  GemmArgs g;
  make_gemm_args(L->args, g);
  g.terms = terms;
  g.tscale = scale;
  g.K = n_terms;
  if ((st = run_gemm(c, g, false, res)) != CCUT_OK) return st;
  if (out_stderr_l1) {
    // second moment: res2 = 2^-k sum_j (w_j / (N q_j))^2 2^2k, so with
    // Y_j the j-th term of the estimate, sum_j Y_j^2 = 2^-k res2 and the
    // standard error of entry b is sqrt(sum_j Y_j^2 - est_b^2 / N)
    g.square = 1;
    if ((st = run_gemm(c, g, false, res2)) != CCUT_OK) return st;
    std::vector<double> e(bins), e2(bins);
    HIP_TRY(c, hipMemcpyAsync(e.data(), res, bins * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(e2.data(), res2, bins * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    double l1 = 0.0;
    for (uint64_t b = 0; b < bins; ++b)
      l1 += std::sqrt(std::max(0.0, std::ldexp(e2[b], -(int)L->k) - e[b] * e[b] / (double)n_terms));
    *out_stderr_l1 = l1;
  }
  return finish_out(c, res, out, bins, out_on_device);
}

ccut_status ccut_mlp_train_step(ccut_mlp *M, const float *x, const float *t, uint64_t n, float lr, float *loss) {
  if (!M) return CCUT_E_INVALID;
  ccut_ctx *c = M->ctx;
  ccut_status st = begin_call(c);
  if (st != CCUT_OK) return st;
  if (!x || !t) return fail(c, CCUT_E_INVALID, "NULL argument");
  if (n == 0 || n % 64 || n > (1u << 24)) return fail(c, CCUT_E_INVALID, "n must be a positive multiple of 64, at most 2^24");
  if ((st = mlp_ensure_work(M, n)) != CCUT_OK) return st;
  float *lsum = aget<float>(c, 1);
  if (!lsum) return fail(c, CCUT_E_OOM, "device allocation failed");
  // the batch is every row, in order: features rounded to bf16, targets as given
  HIP_TRY(c, launch_to_bf16(x, M->xb, n * M->F, c->stream));
  HIP_TRY(c, hipMemcpyAsync(M->tb, t, n * 4, hipMemcpyDeviceToDevice, c->stream));
  if ((st = mlp_forward_rows(M, M->xb, n, M->y)) != CCUT_OK) return st;
  if ((st = mlp_backward_rows(M, M->xb, M->tb, n, lsum)) != CCUT_OK) return st;
  M->t += 1;
  const float c1 = (float)(1.0 - std::pow(0.9, (double)M->t));
  const float c2 = (float)(1.0 - std::pow(0.999, (double)M->t));
  {
    KTimer tm(c, CCUT_K_MLP);
    HIP_TRY(c, launch_adam(M->p, M->g, M->m, M->v, M->pb, M->n_params, lr, 0.9f, 0.999f, c1, c2, 1e-8f, c->stream));
  }
  if (loss) {
    HIP_TRY(c, hipMemcpyAsync(loss, lsum, 4, hipMemcpyDeviceToHost, c->stream));
    if ((st = sync_call(c)) != CCUT_OK) return st;
    *loss /= (float)n;
    return CCUT_OK;
  }
  return sync_call(c);
}

}  // extern "C"

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
  }
  void *get(size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    if (bytes == 0) bytes = 256;
    for (auto &c : chunks)
      if (c.cap - c.used >= bytes) {
        void *r = c.p + c.used;
        c.used += bytes;
        return r;
      }
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
  hipStream_t stream = nullptr;
  uint32_t max_nc = 12, max_cuts = 12;
  std::string err;
  std::atomic<int> cancel{0};
  Arena arena;
  bool timing = false;
  std::vector<PendingTiming> pending;
  std::vector<hipEvent_t> event_pool;
  uint64_t launches[CCUT_K_COUNT] = {};
  double total_ms[CCUT_K_COUNT] = {};
};

struct ccut_plan {
  ccut_ctx *ctx = nullptr;
  PlanData pd;
  std::vector<uint32_t *> d_ops;   // per fragment, uploaded on first evaluation
  std::vector<double *> d_theta;
  std::vector<size_t> op_bytes;
  ~ccut_plan() {
    for (auto p : d_ops)
      if (p) (void)hipFree(p);
    for (auto p : d_theta)
      if (p) (void)hipFree(p);
  }
};

static thread_local std::string g_create_err;

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
      if (a) (void)hipEventRecord(a, c->stream);
    }
  }
  ~KTimer() {
    if (c->timing && a && b) {
      (void)hipEventRecord(b, c->stream);
      c->pending.push_back({kid, a, b});
    }
  }
};

template <class T>
T *aget(ccut_ctx *c, size_t count) {
  return (T *)c->arena.get(count * sizeof(T));
}

ccut_status ensure_ops(ccut_plan *p) {
  ccut_ctx *c = p->ctx;
  if (!p->d_ops.empty()) return CCUT_OK;
  for (const Fragment &f : p->pd.frags) {
    uint32_t *o = nullptr;
    double *t = nullptr;
    size_t n = std::max<size_t>(f.op_words.size(), 1);
    HIP_TRY(c, hipMalloc(&o, n * sizeof(uint32_t)));
    HIP_TRY(c, hipMalloc(&t, n * sizeof(double)));
    if (!f.op_words.empty()) {
      HIP_TRY(c, hipMemcpy(o, f.op_words.data(), f.op_words.size() * 4, hipMemcpyHostToDevice));
      HIP_TRY(c, hipMemcpy(t, f.op_theta.data(), f.op_theta.size() * 8, hipMemcpyHostToDevice));
    }
    p->d_ops.push_back(o);
    p->d_theta.push_back(t);
  }
  return CCUT_OK;
}

ccut_status check_eval(ccut_plan *p, const ccut_eval_opts *eo) {
  if (!p || !eo) return CCUT_E_INVALID;
  ccut_ctx *c = p->ctx;
  if (c->device < 0) return fail(c, CCUT_E_DEVICE, "host-only context: evaluation needs a device");
  if (eo->precision != CCUT_FP64 && eo->precision != CCUT_FP32_MFMA_FP64SUM)
    return fail(c, CCUT_E_INVALID, "unknown precision mode");
  HIP_TRY(c, hipSetDevice(c->device));
  c->cancel.store(0);
  c->arena.reset();
  return ensure_ops(p);
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

FragDev *upload_frag(ccut_plan *p, const Fragment &f, const FragRequest &r, uint32_t circuit,
                     FragDev &h) {
  ccut_ctx *c = p->ctx;
  h = make_frag_dev(f, r, ((uint64_t)circuit << 40) | ((uint64_t)f.index << 32));
  h.ops = p->d_ops[f.index];
  h.theta = p->d_theta[f.index];
  FragDev *d = aget<FragDev>(c, 1);
  if (!d) return nullptr;
  if (hipMemcpyAsync(d, &h, sizeof(FragDev), hipMemcpyHostToDevice, c->stream) != hipSuccess) return nullptr;
  return d;
}

// Per-variant outcome distributions dist[v][x] over the measured set.
ccut_status variant_dists(ccut_plan *p, const ccut_eval_opts *eo, const Fragment &f,
                          const FragRequest &r, double **dist_out) {
  ccut_ctx *c = p->ctx;
  const uint32_t nm = (uint32_t)r.meas.size();
  const uint64_t nv = f.n_variants;
  if (f.clifford && nm > (uint32_t)kMaxMeas)
    return fail(c, CCUT_E_UNSUPPORTED, "Clifford fragment with more than 64 measured qubits");
  if (nm > (uint32_t)kMaxTableBits)
    return fail(c, CCUT_E_UNSUPPORTED, "outcome table over more than 24 measured qubits");
  if ((nv << nm) > (uint64_t(1) << 34))
    return fail(c, CCUT_E_UNSUPPORTED, "variant tables exceed 2^34 entries");
  FragDev h;
  FragDev *d = upload_frag(p, f, r, eo->circuit, h);
  double *dist = aget<double>(c, nv << nm);
  if (!d || !dist) return fail(c, CCUT_E_OOM, "device allocation failed");
  if (!f.clifford) {
    KTimer t(c, CCUT_K_SV);
    HIP_TRY(c, launch_sv(d, h, 0, nv, dist, c->stream));
  } else {
    uint64_t *models = aget<uint64_t>(c, nv * model_words(nm));
    if (!models) return fail(c, CCUT_E_OOM, "device allocation failed");
    {
      KTimer t(c, CCUT_K_TABLEAU);
      HIP_TRY(c, launch_tableau(d, h, 0, nv, models, c->stream));
    }
    if (eo->shots_per_variant == 0) {
      KTimer t(c, CCUT_K_EXACT);
      HIP_TRY(c, launch_exact_tables(models, nm, nv, dist, c->stream));
    } else {
      const uint64_t shots = eo->shots_per_variant;
      const uint32_t bins = 1u << nm;
      const uint64_t nquads = (shots + 3) / 4;
      for (uint64_t v0 = 0; v0 < nv; v0 += 65535) {
        const uint64_t cnv = std::min<uint64_t>(65535, nv - v0);
        const bool lds = nm <= 14;
        uint32_t nblk = 1;
        if (lds) {
          uint64_t want = (1024 + cnv - 1) / cnv;
          uint64_t maxb = (nquads + 255) / 256;
          nblk = (uint32_t)std::max<uint64_t>(1, std::min(want, maxb));
        } else {
          nblk = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((nquads + 1023) / 1024, 4096));
        }
        const uint32_t qpt = (uint32_t)((nquads + (uint64_t)nblk * 256 - 1) / ((uint64_t)nblk * 256));
        const uint64_t pcount = lds ? cnv * nblk * (uint64_t)bins : cnv * (uint64_t)bins;
        uint32_t *partial = aget<uint32_t>(c, pcount);
        if (!partial) return fail(c, CCUT_E_OOM, "device allocation failed");
        if (!lds) HIP_TRY(c, hipMemsetAsync(partial, 0, pcount * 4, c->stream));
        {
          KTimer t(c, CCUT_K_SAMPLE);
          HIP_TRY(c, launch_sample_hist(models + v0 * model_words(nm), nm, cnv, shots, eo->seed,
                                        h.vid_base + v0, partial, nblk, qpt, nullptr, c->stream));
        }
        {
          KTimer t(c, CCUT_K_HIST_REDUCE);
          HIP_TRY(c, launch_hist_reduce(partial, cnv, lds ? nblk : 1, bins, shots, dist + (v0 << nm),
                                        c->stream));
        }
      }
    }
  }
  *dist_out = dist;
  return cancelled(c);
}

// Per-axis Pauli-basis passes: data[v][x] -> T[p_f][rest], where rest is
// the x part with the output bits removed (mode 1) or the J part consumed
// (mode 2, parity tables laid out [v][J][string]).
ccut_status pauli_passes(ccut_ctx *c, const Fragment &f, const FragRequest &r, double *data,
                         uint64_t xsize, uint64_t mode2_lo, double **out) {
  const uint32_t a = (uint32_t)f.axes.size();
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
      HIP_TRY(c, launch_transform_pass(cur, nxt, outer, R, xsize, lo, mode, c->stream));
    }
    cur = nxt;
    rad[j] = 4;
    xsize = xout;
  }
  *out = cur;
  return CCUT_OK;
}

ccut_status finish_out(ccut_ctx *c, const double *dev, double *out, size_t count, int on_device) {
  HIP_TRY(c, hipMemcpyAsync(out, dev, count * sizeof(double),
                            on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
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

void ccut_ctx_destroy(ccut_ctx *c) {
  if (!c) return;
  if (c->device >= 0) {
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (auto &pt : c->pending) {
      (void)hipEventDestroy(pt.a);
      (void)hipEventDestroy(pt.b);
    }
    for (auto e : c->event_pool) (void)hipEventDestroy(e);
    c->arena.release();
  }
  delete c;
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
  c->err.clear();
  return CCUT_OK;
}

void ccut_plan_destroy(ccut_plan *p) {
  if (p && p->ctx && p->ctx->device >= 0) (void)hipSetDevice(p->ctx->device);
  delete p;
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
  if (fragment >= p->pd.frags.size()) return fail(c, CCUT_E_INVALID, "fragment out of range");
  if ((st = check_request(c, p->pd.n, qubits, nq, p->pd.n)) != CCUT_OK) return st;
  const Fragment &f = p->pd.frags[fragment];
  FragRequest r = marginal_request(f, qubits, nq);
  double *dist = nullptr, *T = nullptr;
  if ((st = variant_dists(p, eo, f, r, &dist)) != CCUT_OK) return st;
  if ((st = pauli_passes(c, f, r, dist, 1ull << r.meas.size(), 0, &T)) != CCUT_OK) return st;
  size_t count = ((size_t)1 << (2 * f.axes.size())) << r.req_pos.size();
  return finish_out(c, T, out, count, on_device);
}

ccut_status ccut_marginal(ccut_plan *p, const ccut_eval_opts *eo, const uint32_t *qubits, uint32_t nq,
                          double *out, int on_device) {
  ccut_status st = check_eval(p, eo);
  if (st != CCUT_OK) return st;
  ccut_ctx *c = p->ctx;
  if (!out) return fail(c, CCUT_E_INVALID, "out is NULL");
  if ((st = check_request(c, p->pd.n, qubits, nq)) != CCUT_OK) return st;
  const PlanData &pd = p->pd;
  if (pd.frags.size() > (size_t)kMaxFrags) return fail(c, CCUT_E_UNSUPPORTED, "more than 64 fragments");
  RecombArgs args{};
  args.n_frags = (uint32_t)pd.frags.size();
  args.k = pd.k;
  for (const Fragment &f : pd.frags) {
    FragRequest r = marginal_request(f, qubits, nq);
    double *dist = nullptr, *T = nullptr;
    if ((st = variant_dists(p, eo, f, r, &dist)) != CCUT_OK) return st;
    if ((st = pauli_passes(c, f, r, dist, 1ull << r.meas.size(), 0, &T)) != CCUT_OK) return st;
    RecombFrag &rf = args.f[f.index];
    rf.T = T;
    rf.n_axes = (uint32_t)f.axes.size();
    rf.rows = 1u << r.req_pos.size();
    rf.n_req = (uint32_t)r.req_pos.size();
    for (size_t j = 0; j < f.axes.size(); ++j) rf.axis_cut[j] = f.axes[j].cut;
    for (size_t i = 0; i < r.req_user.size(); ++i) rf.req_user[i] = r.req_user[i];
    if ((st = cancelled(c)) != CCUT_OK) return st;
  }
  RecombArgs *dargs = aget<RecombArgs>(c, 1);
  double *res = aget<double>(c, (size_t)1 << nq);
  if (!dargs || !res) return fail(c, CCUT_E_OOM, "device allocation failed");
  HIP_TRY(c, hipMemcpyAsync(dargs, &args, sizeof(args), hipMemcpyHostToDevice, c->stream));
  {
    KTimer t(c, CCUT_K_RECOMBINE);
    HIP_TRY(c, launch_recombine_fp64(dargs, nq, res, c->stream));
  }
  return finish_out(c, res, out, (size_t)1 << nq, on_device);
}

ccut_status ccut_zexpect(ccut_plan *p, const ccut_eval_opts *eo, const uint64_t *masks, uint32_t n_strings,
                         double *out, int on_device) {
  ccut_status st = check_eval(p, eo);
  if (st != CCUT_OK) return st;
  ccut_ctx *c = p->ctx;
  if (!out || (n_strings && !masks)) return fail(c, CCUT_E_INVALID, "NULL argument");
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
  for (const Fragment &f : pd.frags) {
    FragRequest r = zstring_request(f, anymask);
    const uint32_t nm = (uint32_t)r.meas.size();
    const uint64_t nv = f.n_variants;
    if (nm > (uint32_t)kMaxMeas) return fail(c, CCUT_E_UNSUPPORTED, "more than 64 measured qubits in a fragment");
    // extended masks [J][string] over measured positions
    std::vector<uint32_t> outpos;
    for (size_t j = 0; j < f.axes.size(); ++j)
      if (f.axes[j].side == 0) outpos.push_back((uint32_t)r.axis_outpos[j]);
    const uint32_t n_out = (uint32_t)outpos.size();
    if (n_out > 12) return fail(c, CCUT_E_UNSUPPORTED, "more than 12 quantum outputs in a fragment");
    const uint32_t n_ext = n_strings << n_out;
    std::vector<uint64_t> ext(n_ext);
    for (uint32_t s = 0; s < n_strings; ++s) {
      uint64_t z = 0;
      for (uint32_t jpos = 0; jpos < nm; ++jpos) {
        const uint32_t wire = f.wires[r.meas[jpos]];
        const bool is_cout = f.out_local[wire] == (int32_t)r.meas[jpos];
        if (is_cout && ((masks[(size_t)s * nw + (wire >> 6)] >> (wire & 63)) & 1ull)) z |= 1ull << jpos;
      }
      for (uint32_t J = 0; J < (1u << n_out); ++J) {
        uint64_t e = z;
        for (uint32_t i = 0; i < n_out; ++i)
          if ((J >> i) & 1u) e |= 1ull << outpos[i];
        ext[(size_t)J * n_strings + s] = e;
      }
    }
    uint64_t *d_ext = aget<uint64_t>(c, n_ext);
    double *E = aget<double>(c, nv * n_ext);
    if (!d_ext || !E) return fail(c, CCUT_E_OOM, "device allocation failed");
    HIP_TRY(c, hipMemcpyAsync(d_ext, ext.data(), n_ext * 8, hipMemcpyHostToDevice, c->stream));
    FragDev h;
    FragDev *d = upload_frag(p, f, r, eo->circuit, h);
    if (!d) return fail(c, CCUT_E_OOM, "device allocation failed");
    if (!f.clifford) {
      double *dist = aget<double>(c, nv << nm);
      if (!dist) return fail(c, CCUT_E_OOM, "device allocation failed");
      {
        KTimer t(c, CCUT_K_SV);
        HIP_TRY(c, launch_sv(d, h, 0, nv, dist, c->stream));
      }
      KTimer t(c, CCUT_K_PARITY);
      HIP_TRY(c, launch_dist_parity(dist, nm, nv, d_ext, n_ext, E, c->stream));
    } else {
      uint64_t *models = aget<uint64_t>(c, nv * model_words(nm));
      if (!models) return fail(c, CCUT_E_OOM, "device allocation failed");
      {
        KTimer t(c, CCUT_K_TABLEAU);
        HIP_TRY(c, launch_tableau(d, h, 0, nv, models, c->stream));
      }
      if (eo->shots_per_variant == 0) {
        KTimer t(c, CCUT_K_PARITY);
        HIP_TRY(c, launch_parity_exact(models, nm, nv, d_ext, n_ext, E, c->stream));
      } else {
        uint32_t *odd = aget<uint32_t>(c, nv * n_ext);
        if (!odd) return fail(c, CCUT_E_OOM, "device allocation failed");
        HIP_TRY(c, hipMemsetAsync(odd, 0, nv * n_ext * 4, c->stream));
        for (uint64_t v0 = 0; v0 < nv; v0 += 65535) {
          const uint64_t cnv = std::min<uint64_t>(65535, nv - v0);
          KTimer t(c, CCUT_K_PARITY);
          HIP_TRY(c, launch_parity_sampled(models + v0 * model_words(nm), nm, cnv, eo->shots_per_variant,
                                           eo->seed, h.vid_base + v0, d_ext, n_ext, odd + v0 * n_ext,
                                           c->stream));
        }
        HIP_TRY(c, launch_parity_finish(odd, nv * n_ext, eo->shots_per_variant, E, c->stream));
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
  RecombArgs *dargs = aget<RecombArgs>(c, 1);
  double *res = aget<double>(c, n_strings);
  if (!dargs || !res) return fail(c, CCUT_E_OOM, "device allocation failed");
  HIP_TRY(c, hipMemcpyAsync(dargs, &args, sizeof(args), hipMemcpyHostToDevice, c->stream));
  {
    KTimer t(c, CCUT_K_ZRECOMBINE);
    HIP_TRY(c, launch_zrecombine_fp64(dargs, n_strings, res, c->stream));
  }
  return finish_out(c, res, out, n_strings, on_device);
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
  if (eo->shots_per_variant == 0) return fail(c, CCUT_E_INVALID, "shot records need shots > 0");
  if (v_begin > v_end || v_end > f.n_variants) return fail(c, CCUT_E_INVALID, "bad variant range");
  const uint64_t nv = v_end - v_begin;
  if (nv == 0) return CCUT_OK;
  FragRequest r = marginal_request(f, qubits, nq);
  const uint32_t nm = (uint32_t)r.meas.size();
  if (nm > (uint32_t)kMaxMeas) return fail(c, CCUT_E_UNSUPPORTED, "more than 64 measured qubits");
  FragDev h;
  FragDev *d = upload_frag(p, f, r, eo->circuit, h);
  uint64_t *models = aget<uint64_t>(c, nv * model_words(nm));
  const uint64_t shots = eo->shots_per_variant;
  uint64_t *rec = aget<uint64_t>(c, nv * shots);
  if (!d || !models || !rec) return fail(c, CCUT_E_OOM, "device allocation failed");
  {
    KTimer t(c, CCUT_K_TABLEAU);
    HIP_TRY(c, launch_tableau(d, h, v_begin, nv, models, c->stream));
  }
  const uint64_t nquads = (shots + 3) / 4;
  for (uint64_t v0 = 0; v0 < nv; v0 += 65535) {
    const uint64_t cnv = std::min<uint64_t>(65535, nv - v0);
    const uint32_t nblk = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((nquads + 255) / 256, 4096));
    const uint32_t qpt = (uint32_t)((nquads + (uint64_t)nblk * 256 - 1) / ((uint64_t)nblk * 256));
    KTimer t(c, CCUT_K_SAMPLE);
    HIP_TRY(c, launch_sample_hist(models + v0 * model_words(nm), nm, cnv, shots, eo->seed,
                                  h.vid_base + v_begin + v0, nullptr, nblk, qpt, rec + v0 * shots, c->stream));
  }
  HIP_TRY(c, hipMemcpyAsync(out, rec, nv * shots * 8, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                            c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
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
  static const char *names[CCUT_K_COUNT] = {"tableau_kernel", "sample_kernel", "hist_reduce_kernel",
                                            "exact_kernel", "sv_kernel", "parity_kernel",
                                            "transform_pass_kernel", "recombine_fp64_kernel",
                                            "zrecombine_fp64_kernel"};
  return kid < CCUT_K_COUNT ? names[kid] : "";
}

}  // extern "C"

// Pauli-basis transform of fragment variant data, and the recombination
// sum over cut terms (the contraction of the paper's Sec. V-C, one tensor
// per fragment and one index per cut).
//
// Transform, per cut axis (wire-cutting identity
// rho = 1/2 sum_P Tr(P rho) P):
//   quantum input, prepared in (0, 1, +, +i):
//     I = p0 + p1, X = 2 p+ - p0 - p1, Y = 2 p+i - p0 - p1, Z = p0 - p1
//   quantum output, measured in basis (X, Y, Z) with outcome bit o:
//     I = Z0 + Z1, X = X0 - X1, Y = Y0 - Y1, Z = Z0 - Z1
// applied one axis at a time; the fragment tensor ends as T_f[p_f][b_f].
#include <algorithm>

#include "common.hpp"

// products and sums exactly as written (no contraction into fma), so every
// kernel that shares a body computes the same bits
#pragma clang fp contract(off)

namespace ccut {

namespace {

inline unsigned blocks_for(uint64_t n, unsigned bs) { return (unsigned)((n + bs - 1) / bs); }

// Layout of the data before the pass: flat = ((o * rin + d) * R + r) * X + x.
// mode 0: input axis (rin = 4); mode 1/2: output axis (rin = 3), its
// outcome (mode 1) or parity-selection (mode 2) bit sits in x at stride lo.
__global__ void transform_pass_kernel(const double *__restrict__ in, double *__restrict__ out,
                                      uint64_t outer, uint64_t R, uint64_t Xin, uint64_t lo, int mode) {
  const uint64_t Xout = mode == 0 ? Xin : Xin / 2;
  const uint64_t total = outer * 4 * R * Xout;
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const uint64_t x = i % Xout;
  const uint64_t r = (i / Xout) % R;
  const uint32_t P = (uint32_t)((i / (Xout * R)) % 4);
  const uint64_t o = i / (Xout * R * 4);
  double acc;
  if (mode == 0) {
    auto at = [&](uint32_t s) { return in[((o * 4 + s) * R + r) * Xin + x]; };
    const double p0 = at(0), p1 = at(1);
    switch (P) {
      case 0: acc = p0 + p1; break;
      case 1: acc = 2.0 * at(2) - p0 - p1; break;
      case 2: acc = 2.0 * at(3) - p0 - p1; break;
      default: acc = p0 - p1; break;
    }
  } else {
    const uint64_t xhi = x / lo, xlo = x % lo;
    const uint64_t x0 = (xhi * 2) * lo + xlo, x1 = x0 + lo;
    const uint32_t basis = (P == 1) ? 0u : (P == 2) ? 1u : 2u;  // X, Y, Z(for I and Z)
    const double *src = in + ((o * 3 + basis) * R + r) * Xin;
    if (mode == 1)
      acc = (P == 0) ? src[x0] + src[x1] : src[x0] - src[x1];
    else
      acc = (P == 0) ? src[x0] : src[x1];
  }
  out[i] = acc;
}

// One thread per output entry; the terms of every axis are enumerated as a
// mixed-radix counter (at most 3 per input axis, 2 or 1 per output axis).
__global__ void transform_all_kernel(const TransformAll A, const double *__restrict__ in, double *__restrict__ out) {
  const uint32_t a = A.n_axes;
  const uint64_t total = (A.x_out << (2 * a));
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const uint64_t x = i % A.x_out;
  const uint64_t P = i / A.x_out;
  // per axis: number of terms and the term list (digit, outcome bit, coefficient)
  uint32_t nt[kMaxAxes];
  for (uint32_t j = 0; j < a; ++j) {
    const uint32_t p = (uint32_t)((P >> (2 * j)) & 3ull);
    nt[j] = A.mode[j] == 0 ? (p == 1 || p == 2 ? 3u : 2u) : A.mode[j] == 1 ? 2u : 1u;
  }
  // x with the consumed outcome bits (mode 1) as zeros, ascending positions
  uint64_t xbase = x;
  if (A.n_strings == 0) {
    uint32_t ps[kMaxAxes], np = 0;
    for (uint32_t j = 0; j < a; ++j)
      if (A.mode[j] == 1) ps[np++] = A.pos[j];
    for (uint32_t u = 1; u < np; ++u)  // insertion sort, np <= 16
      for (uint32_t v = u; v > 0 && ps[v - 1] > ps[v]; --v) {
        const uint32_t t = ps[v];
        ps[v] = ps[v - 1];
        ps[v - 1] = t;
      }
    for (uint32_t u = 0; u < np; ++u)
      xbase = ((xbase >> ps[u]) << (ps[u] + 1)) | (xbase & ((1ull << ps[u]) - 1));
  }
  double acc = 0.0;
  uint32_t c[kMaxAxes];
  for (uint32_t j = 0; j < a; ++j) c[j] = 0;
  for (;;) {
    double coef = 1.0;
    uint64_t v = 0, stride = 1, xin = xbase, J = 0;
    uint32_t t_out = 0;
    for (uint32_t j = 0; j < a; ++j) {
      const uint32_t p = (uint32_t)((P >> (2 * j)) & 3ull);
      uint32_t d, b = 0;
      double w;
      if (A.mode[j] == 0) {
        // I: p0 + p1; X: 2p+ - p0 - p1; Y: 2p+i - p0 - p1; Z: p0 - p1
        if (p == 0) { d = c[j]; w = 1.0; }
        else if (p == 3) { d = c[j]; w = c[j] ? -1.0 : 1.0; }
        else if (c[j] == 0) { d = p + 1; w = 2.0; }
        else { d = c[j] - 1; w = -1.0; }
      } else {
        d = p == 1 ? 0u : p == 2 ? 1u : 2u;  // basis X, Y, Z (I reads Z)
        if (A.mode[j] == 1) {
          b = c[j];
          w = (p != 0 && b) ? -1.0 : 1.0;
        } else {
          b = p == 0 ? 0u : 1u;
          w = 1.0;
        }
        if (A.mode[j] == 1) xin |= (uint64_t)b << A.pos[j];
        else J |= (uint64_t)b << t_out;
        ++t_out;
      }
      coef *= w;
      v += d * stride;
      stride *= A.rad[j];
    }
    if (A.n_strings) xin = J * A.n_strings + x;
    acc += coef * in[v * A.x_in + xin];
    uint32_t j = 0;
    while (j < a && ++c[j] == nt[j]) c[j++] = 0;
    if (j == a) break;
  }
  out[i] = acc;
}

// The per-axis passes on LDS tiles.  Workgroup = one tile of 2^t output
// entries x of one job.  The tile's variant data (every variant digit,
// every outcome bit of the output axes) is staged in LDS as
// s[v][l], v mixed radix over the axes (axis 0 fastest), l the tile's x
// (x_in bits below thr, then the high outcome bits).  Each pass rewrites its
// axis in place, group by group, with the operations of the pass kernel:
// an input axis keeps its four slots (I, X, Y, Z); an output axis reads its
// six (basis X, Y, Z x outcome 0, 1) and leaves I, X, Y in the outcome-0
// slots of bases X, Y, Z and Z in the outcome-1 slot of basis X.
// A workgroup takes `per_wg` consecutive tiles of the launch in turn (fewer,
// longer workgroups: the dispatcher, not the tiles, limits short ones), and
// the workgroups of one XCD take consecutive ranges (xcd_block): the tiles
// of a variant row share its cache lines.
constexpr uint32_t kTileThreads = 256;
__device__ __attribute__((always_inline)) void tile_body(const TileJob &J, uint64_t u, double *s, uint32_t *s_xdep,
                                                         uint32_t (*s_pv)[256]);

__global__ __launch_bounds__(kTileThreads) void transform_tiled_kernel(const TileJob *__restrict__ jobs,
                                                                       uint32_t n_jobs, uint64_t total,
                                                                       uint32_t per_wg) {
  __shared__ double s[kTileElems];
  __shared__ uint32_t s_xdep[1u << kTileMaxT];
  __shared__ uint32_t s_pv[2][256];
  const uint64_t g0 = (uint64_t)xcd_block(blockIdx.x, gridDim.x) * per_wg;
  const uint64_t g1 = g0 + per_wg < total ? g0 + per_wg : total;
  uint32_t jb = find_job(jobs, n_jobs, g0, [](const TileJob &J) { return J.wg0; });
  for (uint64_t g = g0; g < g1; ++g) {
    while (jb + 1 < n_jobs && jobs[jb + 1].wg0 <= g) ++jb;
    if (g > g0) __syncthreads();  // the previous tile's LDS is consumed
    tile_body(jobs[jb], g - jobs[jb].wg0, s, s_xdep, s_pv);
  }
}

// The slot offset of the term digits in one byte of P (axes 4 hi .. 4 hi + 3):
// v part (mixed radix, an output axis' Z on its Z-basis slot) shifted by
// lb, or'ed with the outcome bits the output axes' Z set.  Offsets of the
// two bytes add (their v parts add, their outcome bits are disjoint).
template <uint32_t HI>
__device__ inline uint32_t pv_byte(uint32_t pb, const uint32_t *Rv, const uint32_t *o3, const uint32_t *lq,
                                   uint32_t lb) {
  uint32_t v = 0, l = 0;
#pragma unroll
  for (uint32_t jj = 0; jj < 4; ++jj) {
    const uint32_t j = 4 * HI + jj;
    const uint32_t p = (pb >> (2 * jj)) & 3u;
    const uint32_t z = o3[j] & ((p + 1u) >> 2);  // 1 iff p = 3 on an output axis
    v += (p - 3u * z) * Rv[j];
    l |= z << lq[j];
  }
  return (v << lb) | l;
}

__device__ __attribute__((always_inline)) void tile_body(const TileJob &J, uint64_t u, double *s, uint32_t *s_xdep,
                                                         uint32_t (*s_pv)[256]) {
  static_assert(kTileThreads == 256, "one byte of P per thread in the offset tables");
  const uint32_t tid = threadIdx.x;
  const uint32_t a = J.n_axes, V = J.v_count, lb = J.lbits, t = J.t, thr = J.thr, nh = J.nh;
  const uint32_t XL = 1u << lb, XT = 1u << t;
  // the job's per-axis positions in registers, read once (uniform).  Slots
  // past the job's axes hold 0 and are never selected: the bits and digits
  // they would place are 0, so the index arithmetic below needs no guards.
  uint32_t hp[kMaxTileAxes], xp[kTileMaxT];
#pragma unroll
  for (uint32_t h = 0; h < (uint32_t)kMaxTileAxes; ++h) hp[h] = J.hpos[h];
#pragma unroll
  for (uint32_t i = 0; i < kTileMaxT; ++i) xp[i] = J.xpos[i];
  // the tile's fixed x_in bits: u's bits in the non-outcome positions from
  // thr up, i.e. u << thr with a zero inserted at each outcome position at
  // or above thr (ascending)
  uint64_t base = (uint64_t)u << thr;
#pragma unroll
  for (uint32_t h = 0; h < (uint32_t)kMaxTileAxes; ++h)
    if (h < nh) base = ((base >> hp[h]) << (hp[h] + 1)) | (base & ((1ull << hp[h]) - 1ull));
  for (uint32_t xo = tid; xo < XT; xo += kTileThreads) {
    uint32_t l = 0;
#pragma unroll
    for (uint32_t i = 0; i < kTileMaxT; ++i) l |= ((xo >> i) & 1u) << xp[i];
    s_xdep[xo] = l;
  }
  // per-axis radix products, output flags and outcome positions (slots past
  // the axes: radix 0 -> flag 0, digit always 0), then the two byte tables
  {
    uint32_t Rv[kMaxTileAxes], o3[kMaxTileAxes], lq[kMaxTileAxes];
    uint32_t Rj = 1;
#pragma unroll
    for (uint32_t j = 0; j < (uint32_t)kMaxTileAxes; ++j) {
      Rv[j] = Rj;
      o3[j] = J.rad[j] == 3 ? 1u : 0u;
      lq[j] = J.lpos[j];
      Rj *= J.rad[j] ? J.rad[j] : 1u;
    }
    s_pv[0][tid] = pv_byte<0>(tid, Rv, o3, lq, lb);
    s_pv[1][tid] = pv_byte<1>(tid, Rv, o3, lq, lb);
  }
  const uint32_t lowmask = (1u << thr) - 1u;
  const uint32_t n_el = V << lb;
  // x_in bits of a tile-local index l: bits below thr in place, bit thr + h
  // at the outcome position hp[h] (a bit permutation, so the deposit of
  // disjoint bit sets or's)
  auto dep = [&](uint32_t l) {
    uint64_t x = l & lowmask;
#pragma unroll
    for (uint32_t h = 0; h < (uint32_t)kMaxTileAxes; ++h) x |= (((uint64_t)l >> (thr + h)) & 1ull) << hp[h];
    return x;
  };
  // element e = tid + 256 i has l = (tid mod XL) | ((256 i) mod XL) with
  // disjoint bits: this thread's part is deposited once, the second part
  // (nonzero only when XL > 256) is uniform
  const uint64_t xt = base | dep(tid & (XL - 1u));
  // every element's table index first, then all loads, then the
  // conversions: no load waits on the one before it
  constexpr uint32_t kPer = kTileElems / kTileThreads;
  uint64_t idx[kPer];
#pragma unroll
  for (uint32_t i = 0; i < kPer; ++i) {
    const uint32_t e = tid + i * kTileThreads;
    const uint32_t v = e >> lb;
    uint64_t x = xt;
    if (XL > kTileThreads) x |= dep((i * kTileThreads) & (XL - 1u));
    idx[i] = e < n_el ? (uint64_t)v * J.x_in + x : 0;  // entry 0 stands in for the lanes past the tile
  }
  if (J.in16) {
    const __attribute__((address_space(1))) uint16_t *in16 =
        (const __attribute__((address_space(1))) uint16_t *)J.in16;
    const double inv = 1.0 / J.shots;  // a table entry is count x fl(1/shots)
    uint32_t c[kPer];
#pragma unroll
    for (uint32_t i = 0; i < kPer; ++i) c[i] = in16[idx[i]];
#pragma unroll
    for (uint32_t i = 0; i < kPer; ++i) {
      const uint32_t e = tid + i * kTileThreads;
      if (e < n_el) s[e] = (double)c[i] * inv;
    }
  } else {
    const __attribute__((address_space(1))) double *in = (const __attribute__((address_space(1))) double *)J.in;
    double d[kPer];
#pragma unroll
    for (uint32_t i = 0; i < kPer; ++i) d[i] = in[idx[i]];
#pragma unroll
    for (uint32_t i = 0; i < kPer; ++i) {
      const uint32_t e = tid + i * kTileThreads;
      if (e < n_el) s[e] = d[i];
    }
  }
  __syncthreads();
  uint32_t R = 1;  // product of the radices of the axes below j
  for (uint32_t j = 0; j < a; ++j) {
    const uint32_t S = R << lb;  // slot stride of axis j's digit
    const uint32_t mag = J.rmag[j];
    const uint32_t m1 = mag ? 0u : ~0u;  // R_j = 1 (mag 0): the quotient is the value itself, no branch
    // g = q S + r: q = (g >> lb) / R by multiply-high (exact for g < 2^19)
    auto split = [&](uint32_t g, uint32_t &q, uint32_t &r) {
      const uint32_t gh = g >> lb;
      q = __umulhi(gh, mag) + (gh & m1);
      r = ((gh - q * R) << lb) | (g & (XL - 1u));
    };
    if (J.rad[j] == 4) {
      for (uint32_t g = tid; g < (n_el >> 2); g += kTileThreads) {
        uint32_t q, r;
        split(g, q, r);
        const uint32_t b = q * 4 * S + r;
        const double p0 = s[b], p1 = s[b + S], pp = s[b + 2 * S], pi = s[b + 3 * S];
        s[b] = p0 + p1;
        s[b + S] = 2.0 * pp - p0 - p1;
        s[b + 2 * S] = 2.0 * pi - p0 - p1;
        s[b + 3 * S] = p0 - p1;
      }
    } else {
      const uint32_t lp = J.lpos[j], half = XL >> 1, o1 = 1u << lp;
      for (uint32_t g = tid; g < (V / 3) * half; g += kTileThreads) {
        const uint32_t li = g & (half - 1u), vg = g >> (lb - 1);
        const uint32_t l = ((li >> lp) << (lp + 1)) | (li & (o1 - 1u));
        const uint32_t vq = __umulhi(vg, mag) + (vg & m1);
        const uint32_t b = ((vq * 3 * R + (vg - vq * R)) << lb) | l;
        const double x0 = s[b], x1 = s[b + o1], y0 = s[b + S], y1 = s[b + S + o1];
        const double z0 = s[b + 2 * S], z1 = s[b + 2 * S + o1];
        s[b] = z0 + z1;
        s[b + S] = x0 - x1;
        s[b + 2 * S] = y0 - y1;
        s[b + o1] = z0 - z1;
      }
    }
    R *= J.rad[j];
    __syncthreads();
  }
  // folded axes: the four Pauli slots of the axis rewritten into the
  // preparation basis of the fragment downstream of its cut (the map of
  // launch_fold: s=0: I - X - Y + Z, s=1: I - X - Y - Z, s=+: 2X, s=+i: 2Y)
  if (J.fold) {
    R = 1;
    for (uint32_t j = 0; j < a; ++j) {
      if ((J.fold >> j) & 1u) {
        const uint32_t S = R << lb, mag = J.rmag[j];
        const uint32_t m1 = mag ? 0u : ~0u;
        const uint32_t ngroups = J.rad[j] == 4 ? (n_el >> 2) : (V / 3) * (XL >> 1);
        for (uint32_t g = tid; g < ngroups; g += kTileThreads) {
          uint32_t b, s1, s2, s3;
          if (J.rad[j] == 4) {
            const uint32_t gh = g >> lb, q = __umulhi(gh, mag) + (gh & m1);
            b = q * 4 * S + (((gh - q * R) << lb) | (g & (XL - 1u)));
            s1 = b + S, s2 = b + 2 * S, s3 = b + 3 * S;
          } else {
            const uint32_t lp = J.lpos[j], half = XL >> 1, o1 = 1u << lp;
            const uint32_t li = g & (half - 1u), vg = g >> (lb - 1);
            const uint32_t l = ((li >> lp) << (lp + 1)) | (li & (o1 - 1u));
            const uint32_t vq = __umulhi(vg, mag) + (vg & m1);
            b = ((vq * 3 * R + (vg - vq * R)) << lb) | l;
            s1 = b + S, s2 = b + 2 * S, s3 = b + o1;
          }
          const double vI = s[b], vX = s[s1], vY = s[s2], vZ = s[s3];
          s[b] = ((vI - vX) - vY) + vZ;
          s[s1] = ((vI - vX) - vY) - vZ;
          s[s2] = 2.0 * vX;
          s[s3] = 2.0 * vY;
        }
        __syncthreads();
      }
      R *= J.rad[j];
    }
  }
  // out[P][x_out], P base 4 (axis 0 fastest), x_out = u 2^t + xo: the
  // source slot from the two byte tables (P < 4^a <= 4096) and s_xdep;
  // stored through a global pointer (a generic store would hold up the next
  // LDS read until it completes)
  __attribute__((address_space(1))) double *out = (__attribute__((address_space(1))) double *)J.out;
  const uint64_t x_out = J.x_out, ob = (uint64_t)u << t;
  const uint32_t n_out = XT << (2 * a);
  for (uint32_t e = tid; e < n_out; e += kTileThreads) {
    const uint32_t xo = e & (XT - 1u), P = e >> t;
    const uint32_t off = s_pv[0][P & 255u] + s_pv[1][P >> 8] + s_xdep[xo];
    out[(uint64_t)P * x_out + ob + xo] = s[off];
  }
}

// R[b] = 2^-k sum_P prod_f T_f[p_f(P)][b_f(b)], P ascending, fragments in order.
__global__ void recombine_fp64_kernel(const RecombArgs *__restrict__ A, uint32_t nq,
                                      double *__restrict__ outp) {
  const uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= (1ull << nq)) return;
  const uint32_t nf = A->n_frags, k = A->k;
  uint32_t row[kMaxFrags];
  for (uint32_t f = 0; f < nf; ++f) {
    uint32_t r = 0;
    for (uint32_t i = 0; i < A->f[f].n_req; ++i) r |= (uint32_t)((b >> A->f[f].req_user[i]) & 1ull) << i;
    row[f] = r;
  }
  const uint64_t nterms = 1ull << (2 * k);
  double acc = 0.0;
  for (uint64_t P = 0; P < nterms; ++P) {
    double term = 1.0;
    for (uint32_t f = 0; f < nf; ++f) {
      const RecombFrag &F = A->f[f];
      uint32_t p = 0;
      for (uint32_t j = 0; j < F.n_axes; ++j) p |= (uint32_t)((P >> (2 * F.axis_cut[j])) & 3ull) << (2 * j);
      term *= F.T[(uint64_t)p * F.rows + row[f]];
    }
    acc += term;
  }
  outp[b] = ldexp(acc, -(int)k);
}

// The same for at most 8 fragments, with the same operations in the same
// order: per chunk of 128 terms the column offsets p_f(P) * rows_f are
// computed once per workgroup into LDS, each thread keeps its rows in
// registers, and the term loop is unrolled so the gathers overlap.
constexpr uint32_t kRcFrags = 8, kRcChunk = kRcChunkOut;
typedef const __attribute__((address_space(4))) RecombFrag c_RecombFragK;
// terms: the cut terms to sum (ascending), or null for all 4^k.
__device__ inline void recombine_small_body(const RecombArgs *__restrict__ A, uint32_t nq,
                                            double *__restrict__ outp, uint64_t blk,
                                            const uint64_t *__restrict__ terms = nullptr, uint64_t n_terms = 0) {
  __shared__ uint64_t s_off[kRcFrags][kRcChunk];
  typedef const __attribute__((address_space(4))) RecombArgs c_Args;
  typedef const __attribute__((address_space(1))) double g_f64;
  c_Args *C = (c_Args *)(uint64_t)A;  // uniform descriptors: scalar loads
  const uint32_t tid = threadIdx.x;
  const uint64_t b = blk * kRcChunk + tid;
  const bool live = b < (1ull << nq);
  const uint32_t nf = C->n_frags, k = C->k;
  uint32_t row[kRcFrags];
#pragma unroll
  for (uint32_t f = 0; f < kRcFrags; ++f) {
    uint32_t r = 0;
    if (f < nf)
      for (uint32_t i = 0; i < C->f[f].n_req; ++i) r |= (uint32_t)((b >> C->f[f].req_user[i]) & 1ull) << i;
    row[f] = r;
  }
  // global pointers: the gathers never wait behind the LDS offset reads
  g_f64 *T[kRcFrags];
#pragma unroll
  for (uint32_t f = 0; f < kRcFrags; ++f) T[f] = f < nf ? (g_f64 *)(uint64_t)C->f[f].T + row[f] : nullptr;
  const uint64_t nterms = terms ? n_terms : 1ull << (2 * k);
  double acc = 0.0;
  for (uint64_t P0 = 0; P0 < nterms; P0 += kRcChunk) {
    const uint32_t cn = (uint32_t)(nterms - P0 < kRcChunk ? nterms - P0 : kRcChunk);
    __syncthreads();  // the previous chunk is consumed
    if (tid < cn) {
      const uint64_t P = terms ? terms[P0 + tid] : P0 + tid;
      for (uint32_t f = 0; f < nf; ++f) {
        c_RecombFragK &F = C->f[f];
        uint32_t p = 0;
        for (uint32_t j = 0; j < F.n_axes; ++j) p |= (uint32_t)((P >> (2 * F.axis_cut[j])) & 3ull) << (2 * j);
        s_off[f][tid] = (uint64_t)p * F.rows;
      }
    }
    __syncthreads();
    if (!live) continue;
    // batches of U terms: every gather of the batch issued before the
    // first product (the products and the sum in the same order as one
    // term at a time)
    constexpr uint32_t U = 4;
    for (uint32_t t0 = 0; t0 < cn; t0 += U) {
      double v[U][kRcFrags];
#pragma unroll
      for (uint32_t u = 0; u < U; ++u) {
        const uint32_t t = t0 + u < cn ? t0 + u : t0;
#pragma unroll
        for (uint32_t f = 0; f < kRcFrags; ++f)
          if (f < nf) v[u][f] = T[f][s_off[f][t]];
      }
      __builtin_amdgcn_sched_barrier(0);  // the gathers stay ahead of their uses
#pragma unroll
      for (uint32_t u = 0; u < U; ++u) {
        if (t0 + u >= cn) break;
        double term = 1.0;
#pragma unroll
        for (uint32_t f = 0; f < kRcFrags; ++f)
          if (f < nf) term *= v[u][f];
        acc += term;
      }
    }
  }
  if (live) outp[b] = ldexp(acc, -(int)k);
}

__global__ __launch_bounds__(kRcChunk) void recombine_small_kernel(const RecombArgs *__restrict__ A, uint32_t nq,
                                                                   double *__restrict__ outp) {
  recombine_small_body(A, nq, outp, blockIdx.x);
}

__global__ __launch_bounds__(kRcChunk) void recombine_terms_kernel(const RecombArgs *__restrict__ A, uint32_t nq,
                                                                   const uint64_t *__restrict__ terms,
                                                                   uint64_t n_terms, double *__restrict__ outp) {
  recombine_small_body(A, nq, outp, blockIdx.x, terms, n_terms);
}

// nz[c] = 1 if column c (rows contiguous) holds a nonzero: one wave per column.
__global__ __launch_bounds__(256) void colnz_kernel(const double *__restrict__ T, uint32_t rows, uint64_t cols,
                                                    uint8_t *__restrict__ nz) {
  const uint64_t col = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const uint32_t lane = threadIdx.x & 63u;
  if (col >= cols) return;
  const double *c = T + col * rows;
  bool any = false;
  for (uint32_t r = lane; r < rows; r += 64) any |= c[r] != 0.0;
  const uint64_t b = __ballot(any);
  if (lane == 0) nz[col] = b ? 1 : 0;
}

// pos[P] = 1 if every fragment's column p_f(P) is nonzero, else 0.
__global__ void support_flags_kernel(const RecombArgs *__restrict__ A, const SupportArgs sa,
                                     const uint8_t *__restrict__ nz, uint64_t K, uint64_t *__restrict__ pos) {
  const uint64_t P = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (P >= K) return;
  uint64_t f = 1;
  for (uint32_t i = 0; i < A->n_frags && f; ++i) {
    const RecombFrag &F = A->f[i];
    uint64_t p = 0;
    for (uint32_t j = 0; j < F.n_axes; ++j) p |= ((P >> (2 * F.axis_cut[j])) & 3ull) << (2 * j);
    f = nz[sa.off[i] + p];
  }
  pos[P] = f;
}

// after the inclusive scan: term P with flag 1 goes to terms[pos[P] - 1]
__global__ void support_scatter_terms_kernel(const uint64_t *__restrict__ pos, uint64_t K,
                                             uint64_t *__restrict__ terms) {
  const uint64_t P = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (P >= K) return;
  const uint64_t prev = P ? pos[P - 1] : 0;
  if (pos[P] != prev) terms[prev] = P;
}

// Copies of many result vectors in one launch: workgroup (x, y) moves
// elements [x * kGatherChunk, (x + 1) * kGatherChunk) of copy y.
constexpr uint32_t kGatherPer = 4, kGatherChunk = 256 * kGatherPer;
__global__ __launch_bounds__(256) void gather_f64_kernel(const OutCopy *__restrict__ jobs) {
  const OutCopy &J = jobs[blockIdx.y];
  const uint64_t n = J.n, base = (uint64_t)blockIdx.x * kGatherChunk;
  if (base >= n) return;
  const double *src = J.src;
  double *dst = J.dst;
  double v[kGatherPer];
#pragma unroll
  for (uint32_t k = 0; k < kGatherPer; ++k) {
    const uint64_t i = base + k * 256 + threadIdx.x;
    v[k] = i < n ? src[i] : 0.0;
  }
#pragma unroll
  for (uint32_t k = 0; k < kGatherPer; ++k) {
    const uint64_t i = base + k * 256 + threadIdx.x;
    if (i < n) dst[i] = v[k];
  }
}

// Many plans' plain recombinations in one launch.
__global__ __launch_bounds__(kRcChunk) void recombine_batch_kernel(const RcJob *__restrict__ jobs, uint32_t n_jobs) {
  const uint32_t j = find_job(jobs, n_jobs, blockIdx.x, [](const RcJob &J) { return J.wg0; });
  recombine_small_body(jobs[j].args, jobs[j].nq, *jobs[j].out, blockIdx.x - jobs[j].wg0);
}

// <Z_z>[s] = 2^-k sum_P prod_f t_f[p_f(P)][s].  fp64: products and sum in
// fp64, P ascending.  fp32: factors rounded to fp32 and multiplied in fp32
// (with lo_parts: every factor split into fp32 parts t = hi + lo and the
// product taken to first order, prod hi + sum_f lo_f prod_{g!=f} hi_g),
// summed in fp32 over 8 consecutive terms, those sums added in fp64.
template <bool F32>
__global__ void zrecombine_kernel(const RecombArgs *__restrict__ A, uint32_t n_strings, uint64_t per_split,
                                  double *__restrict__ partial) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_strings) return;
  const uint32_t nf = A->n_frags, k = A->k;
  const uint64_t nterms = 1ull << (2 * k);
  const uint64_t P0 = (uint64_t)blockIdx.y * per_split;
  const uint64_t P1 = P0 + per_split < nterms ? P0 + per_split : nterms;
  double acc = 0.0;
  float chunk = 0.f;
  for (uint64_t P = P0; P < P1; ++P) {
    double term = 1.0;
    float hi = 1.f, corr = 0.f;
    for (uint32_t f = 0; f < nf; ++f) {
      const RecombFrag &F = A->f[f];
      uint32_t p = 0;
      for (uint32_t j = 0; j < F.n_axes; ++j) p |= (uint32_t)((P >> (2 * F.axis_cut[j])) & 3ull) << (2 * j);
      const double t = F.T[(uint64_t)p * F.rows + s];
      if (F32) {
        const float th = (float)t, tl = A->lo_parts ? (float)(t - (double)th) : 0.f;
        corr = corr * th + hi * tl;
        hi *= th;
      } else {
        term *= t;
      }
    }
    if (F32) {
      chunk += hi + corr;
      if ((P & 7) == 7 || P + 1 == P1) {
        acc += (double)chunk;
        chunk = 0.f;
      }
    } else {
      acc += term;
    }
  }
  partial[(uint64_t)blockIdx.y * n_strings + s] = acc;
}

// The same for at most 8 fragments (same operations, same order): the
// column offsets of each chunk of 64 terms are computed once per workgroup
// into LDS; with a single term range the result is written directly
// (scaled by 2^-k) and no final pass is needed.
template <bool F32>
__global__ __launch_bounds__(64) void zrecombine_small_kernel(const RecombArgs *__restrict__ A, uint32_t n_strings,
                                                              uint64_t per_split, double *__restrict__ partial,
                                                              double *__restrict__ direct) {
  __shared__ uint64_t s_off[kRcFrags][64];
  typedef const __attribute__((address_space(4))) RecombArgs c_Args;
  typedef const __attribute__((address_space(1))) double g_f64;
  c_Args *C = (c_Args *)(uint64_t)A;  // uniform descriptors: scalar loads
  const uint32_t tid = threadIdx.x;
  const uint32_t s = blockIdx.x * 64 + tid;
  const bool live = s < n_strings;
  const uint32_t nf = C->n_frags, k = C->k, lo_parts = C->lo_parts;
  g_f64 *T[kRcFrags];
#pragma unroll
  for (uint32_t f = 0; f < kRcFrags; ++f) T[f] = f < nf ? (g_f64 *)(uint64_t)C->f[f].T + s : nullptr;
  const uint64_t nterms = 1ull << (2 * k);
  const uint64_t P0 = (uint64_t)blockIdx.y * per_split;
  const uint64_t P1 = P0 + per_split < nterms ? P0 + per_split : nterms;
  double acc = 0.0;
  float chunk = 0.f;
  for (uint64_t C0 = P0; C0 < P1; C0 += 64) {
    const uint32_t cn = (uint32_t)(P1 - C0 < 64 ? P1 - C0 : 64);
    __syncthreads();  // the previous chunk is consumed
    if (tid < cn) {
      const uint64_t P = C0 + tid;
      for (uint32_t f = 0; f < nf; ++f) {
        c_RecombFragK &F = C->f[f];
        uint32_t p = 0;
        for (uint32_t j = 0; j < F.n_axes; ++j) p |= (uint32_t)((P >> (2 * F.axis_cut[j])) & 3ull) << (2 * j);
        s_off[f][tid] = (uint64_t)p * F.rows;
      }
    }
    __syncthreads();
    if (!live) continue;
    constexpr uint32_t U = 4;
    for (uint32_t t0 = 0; t0 < cn; t0 += U) {
      double v[U][kRcFrags];
#pragma unroll
      for (uint32_t u = 0; u < U; ++u) {
        const uint32_t t = t0 + u < cn ? t0 + u : t0;
#pragma unroll
        for (uint32_t f = 0; f < kRcFrags; ++f)
          if (f < nf) v[u][f] = T[f][s_off[f][t]];
      }
      __builtin_amdgcn_sched_barrier(0);  // the gathers stay ahead of their uses
#pragma unroll
      for (uint32_t u = 0; u < U; ++u) {
        if (t0 + u >= cn) break;
        const uint64_t P = C0 + t0 + u;
        double term = 1.0;
        float hi = 1.f, corr = 0.f;
#pragma unroll
        for (uint32_t f = 0; f < kRcFrags; ++f) {
          if (f >= nf) continue;
          const double x = v[u][f];
          if (F32) {
            const float th = (float)x, tl = lo_parts ? (float)(x - (double)th) : 0.f;
            corr = corr * th + hi * tl;
            hi *= th;
          } else {
            term *= x;
          }
        }
        if (F32) {
          chunk += hi + corr;
          if ((P & 7) == 7 || P + 1 == P1) {
            acc += (double)chunk;
            chunk = 0.f;
          }
        } else {
          acc += term;
        }
      }
    }
  }
  if (!live) return;
  if (direct)
    direct[s] = ldexp(acc, -(int)k);
  else
    partial[(uint64_t)blockIdx.y * n_strings + s] = acc;
}

// out[s] = 2^-k sum over term ranges in order
__global__ void zrecombine_final_kernel(const double *__restrict__ partial, uint32_t n_strings, uint32_t splits,
                                        uint32_t k, double *__restrict__ outp) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_strings) return;
  double acc = 0.0;
  for (uint32_t sp = 0; sp < splits; ++sp) acc += partial[(uint64_t)sp * n_strings + s];
  outp[s] = ldexp(acc, -(int)k);
}

}  // namespace

namespace {
// A fragment tensor T[p_f][row] rewritten in place along the marked cut
// axes from the Pauli basis to the preparation basis (0, 1, +, +i) of the
// fragment downstream of that cut: new[s] = sum_P c(P, s) T[P] with the
// input coefficients c (I = p0 + p1, Z = p0 - p1, X = 2p+ - p0 - p1,
// Y = 2p+i - p0 - p1), i.e. s=0: I - X - Y + Z, s=1: I - X - Y - Z,
// s=+: 2X, s=+i: 2Y.  Moving the input coefficients across the sum over
// the cut's Pauli lets the downstream fragment's variant tables stand in
// for its Pauli-basis tensor.  One workgroup per tensor, axis by axis.
__global__ __launch_bounds__(1024) void fold_kernel(const FoldJob *__restrict__ jobs) {
  const FoldJob J = jobs[blockIdx.x];
  const uint64_t fibers = (J.rows << (2 * J.n_axes)) / 4;
  for (uint32_t j = 0; j < J.n_axes; ++j) {
    if (!((J.mask >> j) & 1u)) continue;
    const uint64_t stride = J.rows << (2 * j);  // distance between the P digits of axis j
    for (uint64_t t = threadIdx.x; t < fibers; t += blockDim.x) {
      const uint64_t lo = t % stride, hi = t / stride;
      double *q = J.T + hi * 4 * stride + lo;
      const double vI = q[0], vX = q[stride], vY = q[2 * stride], vZ = q[3 * stride];
      q[0] = ((vI - vX) - vY) + vZ;
      q[stride] = ((vI - vX) - vY) - vZ;
      q[2 * stride] = 2.0 * vX;
      q[3 * stride] = 2.0 * vY;
    }
    __syncthreads();  // the next axis reads what this one wrote
  }
}
}  // namespace

hipError_t launch_fold(const FoldJob *d_jobs, uint32_t n_jobs, hipStream_t s) {
  if (n_jobs == 0) return hipSuccess;
  hipLaunchKernelGGL(fold_kernel, dim3(n_jobs), dim3(1024), 0, s, d_jobs);
  return hipGetLastError();
}

hipError_t launch_transform_pass(const double *in, double *out, uint64_t outer, uint64_t R, uint64_t Xin,
                                 uint64_t lo, int mode, hipStream_t s) {
  const uint64_t Xout = mode == 0 ? Xin : Xin / 2;
  const uint64_t total = outer * 4 * R * Xout;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(transform_pass_kernel, dim3(blocks_for(total, 256)), dim3(256), 0, s, in, out, outer, R,
                     Xin, lo, mode);
  return hipGetLastError();
}

hipError_t launch_transform_all(const TransformAll &a, const double *in, double *out, hipStream_t s) {
  if (a.n_axes == 0 || a.n_axes > (uint32_t)kMaxAxes) return hipErrorInvalidValue;
  const uint64_t total = a.x_out << (2 * a.n_axes);
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(transform_all_kernel, dim3(blocks_for(total, 256)), dim3(256), 0, s, a, in, out);
  return hipGetLastError();
}

hipError_t launch_recombine_fp64(const RecombArgs *d_args, uint32_t n_frags, uint32_t nq, double *out,
                                 hipStream_t s) {
  const uint64_t n = 1ull << nq;
  if (n_frags <= kRcFrags)
    hipLaunchKernelGGL(recombine_small_kernel, dim3(blocks_for(n, kRcChunk)), dim3(kRcChunk), 0, s, d_args, nq, out);
  else
    hipLaunchKernelGGL(recombine_fp64_kernel, dim3(blocks_for(n, 128)), dim3(128), 0, s, d_args, nq, out);
  return hipGetLastError();
}

hipError_t launch_recombine_terms(const RecombArgs *d_args, uint32_t nq, const uint64_t *terms, uint64_t n_terms,
                                  double *out, hipStream_t s) {
  const uint64_t n = 1ull << nq;
  hipLaunchKernelGGL(recombine_terms_kernel, dim3(blocks_for(n, kRcChunk)), dim3(kRcChunk), 0, s, d_args, nq, terms,
                     n_terms, out);
  return hipGetLastError();
}

hipError_t launch_colnz(const double *T, uint32_t rows, uint64_t cols, uint8_t *nz, hipStream_t s) {
  if (cols == 0) return hipSuccess;
  if ((cols + 3) / 4 > 0x7FFFFFFFull) return hipErrorInvalidValue;
  hipLaunchKernelGGL(colnz_kernel, dim3((unsigned)((cols + 3) / 4)), dim3(256), 0, s, T, rows, cols, nz);
  return hipGetLastError();
}

hipError_t launch_gather_f64(const OutCopy *d_jobs, uint32_t n_jobs, uint64_t max_n, hipStream_t s) {
  if (n_jobs == 0 || max_n == 0) return hipSuccess;
  const uint64_t gx = (max_n + kGatherChunk - 1) / kGatherChunk;
  if (n_jobs > 65535u || gx > 0x7FFFFFFFull) return hipErrorInvalidValue;
  hipLaunchKernelGGL(gather_f64_kernel, dim3((unsigned)gx, n_jobs), dim3(256), 0, s, d_jobs);
  return hipGetLastError();
}

hipError_t launch_support_terms(const RecombArgs *d_args, const SupportArgs &sa, const uint8_t *nz, uint64_t K,
                                uint64_t *pos, uint64_t *scratch, uint64_t *terms, hipStream_t s) {
  hipLaunchKernelGGL(support_flags_kernel, dim3(blocks_for(K, 256)), dim3(256), 0, s, d_args, sa, nz, K, pos);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = launch_scan_u64(pos, K, scratch, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(support_scatter_terms_kernel, dim3(blocks_for(K, 256)), dim3(256), 0, s, pos, K, terms);
  return hipGetLastError();
}

hipError_t launch_recombine_batch(const RcJob *d_jobs, uint32_t n_jobs, uint64_t total_wg, hipStream_t s) {
  if (n_jobs == 0 || total_wg == 0) return hipSuccess;
  if (total_wg > 0x7FFFFFFFull) return hipErrorInvalidValue;
  hipLaunchKernelGGL(recombine_batch_kernel, dim3((unsigned)total_wg), dim3(kRcChunk), 0, s, d_jobs, n_jobs);
  return hipGetLastError();
}

hipError_t launch_transform_tiled(const TileJob *d_jobs, uint32_t n_jobs, uint64_t total_tiles, hipStream_t s) {
  if (n_jobs == 0 || total_tiles == 0) return hipSuccess;
  // about 4096 workgroups, at most 16 tiles each
  const uint32_t per_wg = (uint32_t)std::min<uint64_t>(16, std::max<uint64_t>(1, total_tiles / 4096));
  const uint64_t wgs = (total_tiles + per_wg - 1) / per_wg;
  if (wgs > 0x7FFFFFFFull) return hipErrorInvalidValue;
  hipLaunchKernelGGL(transform_tiled_kernel, dim3((unsigned)wgs), dim3(kTileThreads), 0, s, d_jobs, n_jobs,
                     total_tiles, per_wg);
  return hipGetLastError();
}

// term ranges of 64 terms or more (multiples of 8, so fp32 groups never
// straddle a range), about 1024 workgroups in all
uint32_t zrecombine_splits(uint32_t k, uint32_t n_strings) {
  const uint64_t nterms = 1ull << (2 * k);
  const uint64_t sblocks = (n_strings + 63) / 64;
  uint64_t sp = std::max<uint64_t>(1, 1024 / std::max<uint64_t>(sblocks, 1));
  sp = std::min<uint64_t>(sp, (nterms + 63) / 64);
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(sp, 65535));
}

hipError_t launch_zrecombine(const RecombArgs *d_args, uint32_t n_frags, uint32_t k, uint32_t n_strings, bool fp32,
                             double *partial, uint32_t splits, double *out, hipStream_t s) {
  const uint64_t nterms = 1ull << (2 * k);
  uint64_t per = (nterms + splits - 1) / splits;
  per = (per + 7) & ~7ull;
  const dim3 grid(blocks_for(n_strings, 64), splits);
  if (n_frags <= kRcFrags) {
    double *direct = splits == 1 ? out : nullptr;
    if (fp32)
      hipLaunchKernelGGL(zrecombine_small_kernel<true>, grid, dim3(64), 0, s, d_args, n_strings, per, partial, direct);
    else
      hipLaunchKernelGGL(zrecombine_small_kernel<false>, grid, dim3(64), 0, s, d_args, n_strings, per, partial, direct);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || direct) return e;
    hipLaunchKernelGGL(zrecombine_final_kernel, dim3(blocks_for(n_strings, 64)), dim3(64), 0, s, partial, n_strings,
                       splits, k, out);
    return hipGetLastError();
  }
  if (fp32)
    hipLaunchKernelGGL((zrecombine_kernel<true>), grid, dim3(64), 0, s, d_args, n_strings, per, partial);
  else
    hipLaunchKernelGGL((zrecombine_kernel<false>), grid, dim3(64), 0, s, d_args, n_strings, per, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(zrecombine_final_kernel, dim3(blocks_for(n_strings, 64)), dim3(64), 0, s, partial, n_strings,
                     splits, k, out);
  return hipGetLastError();
}

}  // namespace ccut

// Shots, exact tables and Z-parity statistics of Clifford variants from
// their affine sample models (x0, randmask, Gcol): shot s of variant vid
// draws u = the Philox bits of its measurement indices and outputs
// x = x0 ^ (xor of Gcol[a] over random a with u_a = 1).
//
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of
// (c0..c3) <- (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)),
// key bumped by the Weyl constants between rounds.  One call yields four
// 32-bit words: four consecutive shots x 32 measurement indices.
#include <algorithm>

#include "common.hpp"

namespace ccut {

namespace {

// Shot-bit words of one quad (4 shots): bits of measurement indices 0..31
// in lo[r], 32..63 in hi[r].
__device__ inline void quad_bits(uint64_t quad, uint64_t vid, uint64_t seed, bool wide,
                                 uint64_t u[4]) {
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  const U4 lo = philox10(0u, (uint32_t)quad, (uint32_t)vid, (uint32_t)(vid >> 32), k0, k1);
  if (wide) {
    const U4 hi = philox10(1u, (uint32_t)quad, (uint32_t)vid, (uint32_t)(vid >> 32), k0, k1);
#pragma unroll
    for (int r = 0; r < 4; ++r) u[r] = (uint64_t)lo.w[r] | ((uint64_t)hi.w[r] << 32);
  } else {
#pragma unroll
    for (int r = 0; r < 4; ++r) u[r] = lo.w[r];
  }
}

constexpr int kSampleBlock = (int)kSampleThreads;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) u32x4 gu32x4;
typedef __attribute__((address_space(1))) u32x2 gu32x2;
typedef __attribute__((address_space(1))) f64x2 gf64x2;
typedef __attribute__((address_space(1))) uint32_t gu32;
typedef __attribute__((address_space(1))) double gf64;

// Shots counted in an LDS histogram with at most 32 measured indices (no
// records, more than 6 random indices): two quads (8 shots) per step from
// two independent Philox calls, every table lookup of the 8 shots issued
// before its first use, then one packed 16-bit count per shot.  LDS words:
// the 32-bit tables at [0, tw) (tw = 256 per group, in the lower half of
// the region sized for 64-bit entries), one dummy word per lane at
// [tw, tw + 64) that shots outside the count add 0 to (no branch per shot),
// the histogram from 2 tw.  G table groups per shot; SLICED: only outcomes
// whose bits above kLdsHistBits equal `slice` count.  The same shots as the
// generic loop (quad (q0 + q) x kSampleBlock + thread), so the same counts.
template <int G, bool SLICED>
__device__ __attribute__((always_inline)) void narrow_lds_shots(uint32_t *lds, uint32_t x0, uint64_t shots,
                                                                uint64_t vid, uint64_t seed, uint64_t q0,
                                                                uint32_t q_end, uint32_t slice) {
  constexpr uint32_t tw = 256u * G;
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  const uint32_t v_lo = (uint32_t)vid, v_hi = (uint32_t)(vid >> 32);
  const uint64_t nquads = (shots + 3) >> 2;
  const uint32_t dummy = tw + (threadIdx.x & 63u);
  for (uint32_t q = 0; q < q_end; q += 2) {
    if ((q0 + q) * kSampleBlock >= nquads) break;  // the whole workgroup is done
    const uint64_t qa = (q0 + q) * kSampleBlock + threadIdx.x, qb = qa + kSampleBlock;
    // shots of each quad inside the count (0-4)
    const uint64_t sa = 4 * qa, sb = 4 * qb;
    const uint32_t na = sa >= shots ? 0u : shots - sa >= 4 ? 4u : (uint32_t)(shots - sa);
    const uint32_t nb = q + 1 >= q_end || sb >= shots ? 0u : shots - sb >= 4 ? 4u : (uint32_t)(shots - sb);
    const U4 wa = philox10(0u, (uint32_t)qa, v_lo, v_hi, k0, k1);
    const U4 wb = philox10(0u, (uint32_t)qb, v_lo, v_hi, k0, k1);
    uint32_t t[8][G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        t[r][g] = lds[(g << 8) | ((wa.w[r] >> (8 * g)) & 255u)];
        t[4 + r][g] = lds[(g << 8) | ((wb.w[r] >> (8 * g)) & 255u)];
      }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      uint32_t x = x0;
#pragma unroll
      for (int g = 0; g < G; ++g) x ^= t[i][g];
      bool valid = i < 4 ? (uint32_t)i < na : (uint32_t)(i - 4) < nb;
      if (SLICED) {
        valid = valid && (x >> kLdsHistBits) == slice;
        x &= (1u << kLdsHistBits) - 1u;
      }
      const uint32_t w = valid ? 2 * tw + (x >> 1) : dummy;
      atomicAdd(&lds[w], valid ? 1u << (16 * (x & 1u)) : 0u);
    }
  }
}

// Shots of variant v, block bx of nbx: each thread handles `qpt` quads;
// quads are interleaved across the workgroup so record writes are
// contiguous.  With n_meas <= kLdsHistBits (or a slice of the bins) the
// block's histogram lives in LDS as packed 16-bit counts (qpt <= kMaxUnitQpt)
// and is written to partial[v][bx][bins], or straight to the table;
// otherwise counts go to partial[v][bins] (zeroed beforehand).
//
// The xor over random measurements goes by bytes of the Philox word: table
// T[g][b] (LDS, 256 entries per group of 8 measurement indices) holds the
// xor of Gcol[8 g + i] over the bits i of b whose measurement is random, so
// a shot takes ceil(n_meas / 8) lookups.  Dynamic LDS: the tables, then the
// histogram.
__device__ __attribute__((always_inline)) void sample_body(const uint64_t *__restrict__ models, uint32_t n_meas, uint64_t shots, uint64_t seed,
                            uint64_t vid0, uint32_t *__restrict__ partial, uint32_t qpt,
                            uint64_t *__restrict__ records, uint64_t v, uint32_t bx, uint32_t nbx,
                            uint64_t *s_dyn, uint64_t *s_model, uint32_t slice = 0, uint32_t nslice = 1,
                            double *__restrict__ dist = nullptr, uint16_t *__restrict__ cnt16 = nullptr,
                            bool skip = false) {
  const uint32_t mw = model_words(n_meas);
  const uint64_t *md = models + v * mw;
  const uint32_t groups = sample_tab_groups(n_meas);
  uint64_t *s_tab = s_dyn;
  uint32_t *s_hist = reinterpret_cast<uint32_t *>(s_dyn + groups * 256);
  // the model to LDS in one coalesced load, then the tables from LDS
  if (threadIdx.x < mw) s_model[threadIdx.x] = md[threadIdx.x];
  __syncthreads();
  const uint64_t x0 = s_model[0], rmask = s_model[1];
  const uint32_t bins = 1u << n_meas;
  // sliced (nslice > 1): this workgroup counts the outcomes whose top bits
  // equal `slice` into an LDS histogram of 2^kLdsHistBits bins
  const bool sliced = nslice > 1;
  // dist (one shot block): the workgroup writes the table itself, count x fl(1/shots)
  const bool lds_hist = (partial != nullptr || dist != nullptr || cnt16 != nullptr) && (n_meas <= kLdsHistBits || sliced);
  const bool wide = n_meas > 32;
  // With few random bits the shots of a wave land on few bins: lanes with
  // equal outcomes then add their count once (one atomic per distinct
  // outcome in the wave instead of up to 64 on one address).
  const bool combine = (lds_hist || partial != nullptr) && __popcll(rmask) <= 6;
  const bool fast = lds_hist && !wide && records == nullptr && !combine &&
                    ((!sliced && groups >= 1 && groups <= 2) || (sliced && groups == 3));
  uint32_t *s_tab32 = reinterpret_cast<uint32_t *>(s_dyn);  // the fast path's 32-bit entries
  for (uint32_t e = threadIdx.x; e < groups * 256; e += kSampleBlock) {
    const uint32_t g = e >> 8, b = e & 255u;
    uint64_t t = 0;
#pragma unroll
    for (uint32_t i = 0; i < 8; ++i) {
      const uint32_t a = 8 * g + i;
      if (((b >> i) & 1u) && a < n_meas && ((rmask >> a) & 1ull)) t ^= s_model[2 + a];
    }
    if (fast)
      s_tab32[e] = (uint32_t)t;  // at most 32 measured indices: the entry fits
    else
      s_tab[e] = t;
  }
  const uint32_t lbins = sliced ? (1u << kLdsHistBits) : bins;
  const uint32_t lwords = (lbins + 1) / 2;  // two 16-bit counts per word
  if (lds_hist) {
    if (lwords % 4 == 0) {  // 16 bytes per store (the histogram starts 16-byte aligned)
      u32x4 *h4 = reinterpret_cast<u32x4 *>(s_hist);
      for (uint32_t i = threadIdx.x; i < lwords / 4; i += kSampleBlock) h4[i] = u32x4{0u, 0u, 0u, 0u};
    } else {
      for (uint32_t i = threadIdx.x; i < lwords; i += kSampleBlock) s_hist[i] = 0;
    }
  }
  __syncthreads();
  const uint64_t vid = vid0 + v;
  const uint64_t nquads = (shots + 3) >> 2;
  const uint32_t lane = threadIdx.x & 63u;
  uint32_t *hist = lds_hist ? s_hist : (partial ? partial + v * (uint64_t)bins : nullptr);
  // a skipped variant draws no shots: its (zero) histogram is still written
  const uint32_t q_end = skip ? 0u : qpt;
  if (fast) {
    const uint64_t q0 = (uint64_t)bx * qpt;
    if (groups == 1)
      narrow_lds_shots<1, false>(s_tab32, (uint32_t)x0, shots, vid, seed, q0, q_end, slice);
    else if (groups == 2)
      narrow_lds_shots<2, false>(s_tab32, (uint32_t)x0, shots, vid, seed, q0, q_end, slice);
    else
      narrow_lds_shots<3, true>(s_tab32, (uint32_t)x0, shots, vid, seed, q0, q_end, slice);
  }
  for (uint32_t q = 0; q < (fast ? 0u : q_end); ++q) {
    const uint64_t quad = ((uint64_t)bx * qpt + q) * kSampleBlock + threadIdx.x;
    if (!combine && quad >= nquads) break;
    if (combine && ((uint64_t)bx * qpt + q) * kSampleBlock >= nquads) break;  // the whole workgroup is done
    uint64_t u[4];
    quad_bits(quad, vid, seed, wide, u);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const uint64_t s = quad * 4 + r;
      bool valid = quad < nquads && s < shots;
      if (!combine && !valid) break;
      uint64_t x = x0;
      for (uint32_t g = 0; g < groups; ++g) x ^= s_tab[(g << 8) | (uint32_t)((u[r] >> (8 * g)) & 255u)];
      if (records && valid) records[v * shots + s] = x;
      if (sliced) {
        if ((uint32_t)(x >> kLdsHistBits) != slice) valid = false;
        x &= (1u << kLdsHistBits) - 1u;
        if (!combine && !valid) continue;
      }
      if (combine) {
        // every lane of the wave is here (no early exit on this path)
        uint64_t todo = __ballot(valid);
        while (todo) {
          const uint32_t leader = (uint32_t)__ffsll((unsigned long long)todo) - 1u;
          const uint32_t xl = __builtin_amdgcn_readlane((uint32_t)x, leader);
          const uint64_t same = __ballot(valid && (uint32_t)x == xl) & todo;
          if (lane == leader) {
            if (lds_hist)
              atomicAdd(&hist[xl >> 1], (uint32_t)__popcll(same) << (16 * (xl & 1u)));
            else
              atomicAdd(&hist[xl], (uint32_t)__popcll(same));
          }
          todo &= ~same;
        }
      } else if (lds_hist) {
        atomicAdd(&hist[(uint32_t)x >> 1], 1u << (16 * ((uint32_t)x & 1u)));
      } else if (hist) {
        atomicAdd(&hist[x], 1u);
      }
    }
  }
  if (lds_hist) {
    __syncthreads();
    auto count = [&](uint32_t i) { return (s_hist[i >> 1] >> (16 * (i & 1u))) & 0xFFFFu; };
    // Stores go through global pointers (a generic store also counts against
    // the LDS wait counter, so the next LDS read would wait for it).  With at
    // least 8 bins every row starts 16-byte aligned: 16 bytes per store.
    if (cnt16) {
      uint16_t *dd = cnt16 + v * (uint64_t)bins + (uint64_t)slice * lbins;
      if (lbins >= 8) {  // the packed words are the table's layout (little-endian pairs)
        gu32x4 *dst = (gu32x4 *)(dd);
        const u32x4 *src = reinterpret_cast<const u32x4 *>(s_hist);
#pragma unroll 4
        for (uint32_t i = threadIdx.x; i < lwords / 4; i += kSampleBlock) dst[i] = src[i];
      } else if (lbins >= 2) {
        gu32 *dw = (gu32 *)(dd);
        for (uint32_t i = threadIdx.x; i < lwords; i += kSampleBlock) dw[i] = s_hist[i];
      } else if (threadIdx.x == 0) {
        dd[0] = (uint16_t)count(0);
      }
    } else if (dist) {
      double *dd = dist + v * (uint64_t)bins + (uint64_t)slice * lbins;
      const double inv = 1.0 / (double)shots;  // an entry is count x fl(1/shots)
      if (lbins >= 8) {  // one packed word: two entries, 16 bytes
        gf64x2 *dst = (gf64x2 *)(dd);
#pragma unroll 4
        for (uint32_t w = threadIdx.x; w < lwords; w += kSampleBlock) {
          const uint32_t c = s_hist[w];
          dst[w] = f64x2{(double)(c & 0xFFFFu) * inv, (double)(c >> 16) * inv};
        }
      } else {
        gf64 *dst = (gf64 *)(dd);
        for (uint32_t i = threadIdx.x; i < lbins; i += kSampleBlock) dst[i] = (double)(uint64_t)count(i) * inv;
      }
    } else {
      uint32_t *dp = partial + (v * nbx + bx) * (uint64_t)bins + (uint64_t)slice * lbins;
      if (lbins >= 8) {  // one packed word: two counts, 8 bytes
        gu32x2 *dst = (gu32x2 *)(dp);
        for (uint32_t w = threadIdx.x; w < lwords; w += kSampleBlock) {
          const uint32_t c = s_hist[w];
          dst[w] = u32x2{c & 0xFFFFu, c >> 16};
        }
      } else {
        gu32 *dst = (gu32 *)(dp);
        for (uint32_t i = threadIdx.x; i < lbins; i += kSampleBlock) dst[i] = count(i);
      }
    }
  }
}

// grid: (nblk_x, nv)
// vmask (optional): variant v draws its shots only if vmask[v] != 0; the
// others keep all-zero counts (variants no supported cut term reads)
__global__ __launch_bounds__(kSampleBlock) void sample_kernel(
    const uint64_t *__restrict__ models, uint32_t n_meas, uint64_t shots, uint64_t seed,
    uint64_t vid0, uint32_t *__restrict__ partial, uint32_t qpt, uint64_t *__restrict__ records,
    const uint8_t *__restrict__ vmask) {
  extern __shared__ __align__(16) uint64_t s_dyn[];
  __shared__ uint64_t s_model[2 + kMaxMeas];
  const bool skip = vmask && !vmask[blockIdx.y];
  sample_body(models, n_meas, shots, seed, vid0, partial, qpt, records, blockIdx.y, blockIdx.x, gridDim.x, s_dyn,
              s_model, 0, 1, nullptr, nullptr, skip);
}

// Many fragments' sampling in one launch: unit g of the job holding it is
// ((variant x nblk + block) x nslice + slice) = g - wg0, and a workgroup
// takes `per_wg` consecutive units in turn.
__global__ __launch_bounds__(kSampleBlock) void sample_batch_kernel(const SampleJob *__restrict__ jobs,
                                                                      uint32_t n_jobs, uint64_t total,
                                                                      uint32_t per_wg) {
  extern __shared__ __align__(16) uint64_t s_dyn[];
  __shared__ uint64_t s_model[2 + kMaxMeas];
  const uint64_t g0 = (uint64_t)blockIdx.x * per_wg;
  const uint64_t g1 = g0 + per_wg < total ? g0 + per_wg : total;
  uint32_t j = find_job(jobs, n_jobs, g0, [](const SampleJob &J) { return J.wg0; });
  for (uint64_t g = g0; g < g1; ++g) {
    while (j + 1 < n_jobs && jobs[j + 1].wg0 <= g) ++j;
    if (g > g0) __syncthreads();  // the previous unit's tables and histogram are consumed
    const SampleJob &J = jobs[j];
    const uint64_t local = g - J.wg0;
    const uint32_t ns = J.nslice > 1 ? J.nslice : 1u;
    const uint64_t per_v = (uint64_t)J.nblk * ns, rem = local % per_v;
    sample_body(J.models, J.n_meas, J.shots, J.seed, J.vid0, J.partial, J.qpt, nullptr, local / per_v,
                (uint32_t)(rem / ns), J.nblk, s_dyn, s_model, (uint32_t)(rem % ns), ns,
                J.partial || J.cnt16 ? nullptr : J.dist, J.partial ? nullptr : J.cnt16);
  }
}

// dist[v][b] = (sum over shot blocks of counts) x fl(1/shots)
__global__ void hist_reduce_kernel(const uint32_t *__restrict__ partial, uint64_t nv, uint32_t nblk,
                                   uint32_t bins, uint64_t shots, double *__restrict__ dist,
                                   uint16_t *__restrict__ cnt16) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nv * bins) return;
  const uint64_t v = i / bins, b = i % bins;
  uint64_t c = 0;
  for (uint32_t k = 0; k < nblk; ++k) c += partial[(v * nblk + k) * (uint64_t)bins + b];
  if (cnt16)
    cnt16[i] = (uint16_t)c;
  else
    dist[i] = (double)c * (1.0 / (double)shots);  // count x fl(1/shots)
}

// The same over every job of a batch: workgroup x reduces entries
// [(x - rb0) * 4096, ...) of the table of the job holding x (the job lookup
// is done once per workgroup, with uniform loads).
constexpr uint32_t kReduceChunk = 4096;
__global__ __launch_bounds__(256) void hist_reduce_batch_kernel(const SampleJob *__restrict__ jobs, uint32_t n_jobs) {
  const uint32_t j = find_job(jobs, n_jobs, blockIdx.x, [](const SampleJob &J) { return J.rb0; });
  const SampleJob &J = jobs[j];
  const uint32_t bins = 1u << J.n_meas;
  const uint32_t nblk = (J.n_meas <= kLdsHistBits || J.nslice > 1) ? J.nblk : 1u;
  const uint64_t n_e = J.nv * bins;
  const uint64_t e0 = (uint64_t)(blockIdx.x - J.rb0) * kReduceChunk;
  const uint64_t e1 = e0 + kReduceChunk < n_e ? e0 + kReduceChunk : n_e;
  for (uint64_t e = e0 + threadIdx.x; e < e1; e += 256) {
    const uint64_t v = e / bins, b = e % bins;
    uint64_t c = 0;
    for (uint32_t k = 0; k < nblk; ++k) c += J.partial[(v * nblk + k) * (uint64_t)bins + b];
    if (J.cnt16)
      J.cnt16[e] = (uint16_t)c;
    else
      J.dist[e] = (double)c / (double)J.shots;
  }
}

// Exact table: x is an outcome iff y = x ^ x0 equals the xor of the G
// columns of the random measurements a with y_a = 1 (column a of G has
// bit a set and otherwise only bits of later deterministic measurements);
// every outcome has probability 2^-R.
__global__ void exact_kernel(const uint64_t *__restrict__ models, uint32_t n_meas, uint64_t nv,
                             double *__restrict__ dist) {
  const uint64_t bins = 1ull << n_meas;
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nv * bins) return;
  const uint64_t v = i >> n_meas, x = i & (bins - 1);
  const uint64_t *md = models + v * model_words(n_meas);
  const uint64_t rmask = md[1];
  const uint64_t y = x ^ md[0];
  uint64_t e = 0;
  for (uint64_t mm = rmask; mm; mm &= mm - 1) {
    const int a = __ffsll((unsigned long long)mm) - 1;
    if ((y >> a) & 1ull) e ^= md[2 + a];
  }
  const int R = __popcll(rmask);
  dist[i] = (e == y) ? ldexp(1.0, -R) : 0.0;
}

// For mask z over the measured set: z.x = z.x0 ^ g.u with g_a = z.Gcol[a].
__device__ inline void parity_form(const uint64_t *md, uint32_t n_meas, uint64_t z, uint32_t &c,
                                   uint64_t &g) {
  c = __popcll(z & md[0]) & 1u;
  g = 0;
  for (uint32_t a = 0; a < n_meas; ++a) g |= (uint64_t)(__popcll(z & md[2 + a]) & 1) << a;
}

// Exact <(-1)^{z.x}> = (-1)^c if g = 0 else 0 (Clifford expectations are
// -1, 0 or +1).  grid over (v, ext mask).
__global__ void parity_exact_kernel(const uint64_t *__restrict__ models, uint32_t n_meas, uint64_t nv,
                                    const uint64_t *__restrict__ ext, uint32_t n_ext,
                                    double *__restrict__ E) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nv * n_ext) return;
  const uint64_t v = i / n_ext;
  const uint32_t s = (uint32_t)(i % n_ext);
  uint32_t c;
  uint64_t g;
  parity_form(models + v * model_words(n_meas), n_meas, ext[s], c, g);
  E[i] = g ? 0.0 : (c ? -1.0 : 1.0);
}

constexpr int kParityBlock = 256;  // four waves

// Odd-parity counts per (variant, ext mask) over all shots, bit-sliced:
// lane l of a wave owns masks l, 64 + l, ... (G per pass) and the
// wave draws 64 quads (256 shots) per round, one quad per lane.  For shot
// r of every lane, bit j of the 64 random words becomes one 64-bit plane
// (a ballot); a mask's parities over those 64 shots are the XOR of the
// planes of the bits j set in its form g, so one wave instruction serves 64
// shots of 64 masks.  Counts are exact integers.  grid (nblk_x, nv); wave w
// of block x runs rounds [(4x + w) * rounds, (4x + w + 1) * rounds).
template <int kParityGroups>
__global__ __launch_bounds__(kParityBlock) void parity_sampled_kernel(
    const uint64_t *__restrict__ models, uint32_t n_meas, uint64_t shots, uint64_t seed,
    uint64_t vid0, const uint64_t *__restrict__ ext, uint32_t n_ext, uint32_t rounds, uint32_t use_lds,
    uint32_t *__restrict__ odd_counts) {
  extern __shared__ uint32_t s_cnt[];  // [n_ext] per workgroup when use_lds
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t v = blockIdx.y;
  const uint64_t *md = models + v * model_words(n_meas);
  if (use_lds)
    for (uint32_t s = threadIdx.x; s < n_ext; s += kParityBlock) s_cnt[s] = 0;
  __syncthreads();
  const uint64_t vid = vid0 + v;
  const bool wide = n_meas > 32;
  const uint64_t nquads = (shots + 3) >> 2;
  const uint64_t r0 = ((uint64_t)blockIdx.x * (kParityBlock / 64) + wave) * rounds;
  for (uint32_t p0 = 0; p0 < n_ext; p0 += 64 * kParityGroups) {
    uint64_t gm[kParityGroups];
    uint32_t cm[kParityGroups], cnt[kParityGroups];
    uint64_t gall = 0;
#pragma unroll
    for (int k = 0; k < kParityGroups; ++k) {
      const uint32_t s = p0 + 64 * k + lane;
      gm[k] = 0;
      cm[k] = 0;
      cnt[k] = 0;
      if (s < n_ext) parity_form(md, n_meas, ext[s], cm[k], gm[k]);
      gall |= gm[k];
    }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) gall |= __shfl_xor(gall, off);
    gall = __builtin_amdgcn_readfirstlane((uint32_t)gall) |
           ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(gall >> 32)) << 32);
    uint32_t total = 0;  // valid shots seen by this wave
    for (uint32_t rd = 0; rd < rounds; ++rd) {
      const uint64_t quad = (r0 + rd) * 64 + lane;
      uint64_t w[4] = {0, 0, 0, 0};
      if (quad < nquads) quad_bits(quad, vid, seed, wide, w);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint64_t valid = __ballot(quad < nquads && quad * 4 + r < shots);
        if (!valid) continue;
        total += __popcll(valid);
        uint64_t acc[kParityGroups];
#pragma unroll
        for (int k = 0; k < kParityGroups; ++k) acc[k] = 0;
        for (uint64_t rem = gall; rem; rem &= rem - 1) {
          const uint32_t j = (uint32_t)__builtin_ctzll(rem);
          const uint64_t plane = __ballot((w[r] >> j) & 1ull);
#pragma unroll
          for (int k = 0; k < kParityGroups; ++k) acc[k] ^= ((gm[k] >> j) & 1ull) ? plane : 0ull;
        }
#pragma unroll
        for (int k = 0; k < kParityGroups; ++k) cnt[k] += __popcll(acc[k] & valid);
      }
    }
#pragma unroll
    for (int k = 0; k < kParityGroups; ++k) {
      const uint32_t s = p0 + 64 * k + lane;
      const uint32_t odd = cm[k] ? total - cnt[k] : cnt[k];
      if (s < n_ext && odd) atomicAdd(use_lds ? &s_cnt[s] : &odd_counts[v * n_ext + s], odd);
    }
  }
  if (!use_lds) return;
  __syncthreads();
  for (uint32_t s = threadIdx.x; s < n_ext; s += kParityBlock)
    if (s_cnt[s]) atomicAdd(&odd_counts[v * n_ext + s], s_cnt[s]);
}

// settle: a Pauli expectation on a stabilizer state is -1, 0 or +1, so
// shots showing both parities give 0 and shots that agree their sign.
__global__ void parity_finish_kernel(const uint32_t *__restrict__ odd, uint64_t n, uint64_t shots, int settle,
                                     double *__restrict__ E) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (settle)
    E[i] = odd[i] == 0 ? 1.0 : (uint64_t)odd[i] == shots ? -1.0 : 0.0;
  else
    E[i] = ((double)shots - 2.0 * (double)odd[i]) / (double)shots;
}

// <(-1)^{z.x}> for every mask z from an outcome distribution over n_meas
// bits: the Walsh-Hadamard transform W[z] = sum_x (-1)^{z.x} p(x), done in
// place in LDS with n_meas butterfly stages (fixed order, deterministic),
// then gathered at the requested masks.  One workgroup per variant.
constexpr int kWhtBlock = 256;
__global__ __launch_bounds__(kWhtBlock) void dist_parity_kernel(const double *__restrict__ dist, uint32_t n_meas,
                                                                const uint64_t *__restrict__ ext, uint32_t n_ext,
                                                                double *__restrict__ E) {
  extern __shared__ double w[];
  const uint32_t bins = 1u << n_meas;
  const double *p = dist + (uint64_t)blockIdx.x * bins;
  for (uint32_t i = threadIdx.x; i < bins; i += kWhtBlock) w[i] = p[i];
  __syncthreads();
  for (uint32_t s = 0; s < n_meas; ++s) {
    for (uint32_t k = threadIdx.x; k < bins / 2; k += kWhtBlock) {
      const uint32_t i0 = ((k >> s) << (s + 1)) | (k & ((1u << s) - 1)), i1 = i0 | (1u << s);
      const double a = w[i0], b = w[i1];
      w[i0] = a + b;
      w[i1] = a - b;
    }
    __syncthreads();
  }
  double *out = E + (uint64_t)blockIdx.x * n_ext;
  for (uint32_t e = threadIdx.x; e < n_ext; e += kWhtBlock) out[e] = w[ext[e]];
}

inline unsigned blocks_for(uint64_t n, unsigned bs) { return (unsigned)((n + bs - 1) / bs); }

// ------------------------------------------------ more than 64 measurements
// Models of MW words per outcome vector (model_mw): x0[MW], rmask[MW],
// G[a][MW].  Shot bits: measurement index a takes bit a & 31 of Philox
// call a >> 5 (the same draw as below 64).

// The shot words of one quad: u[r][w] = bits 64 w .. 64 w + 63 of shot r.
template <int MW>
__device__ inline void quad_words(uint64_t quad, uint64_t vid, uint64_t seed, uint32_t n_meas, uint64_t (&u)[4][MW]) {
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
  for (int w = 0; w < MW; ++w)
#pragma unroll
    for (int r = 0; r < 4; ++r) u[r][w] = 0;
#pragma unroll
  for (int cidx = 0; cidx < 2 * MW; ++cidx) {
    if ((uint32_t)cidx * 32 >= n_meas) break;
    const U4 o = philox10((uint32_t)cidx, (uint32_t)quad, (uint32_t)vid, (uint32_t)(vid >> 32), k0, k1);
#pragma unroll
    for (int r = 0; r < 4; ++r) u[r][cidx >> 1] |= (uint64_t)o.w[r] << (32 * (cidx & 1));
  }
}

// For a mask z over the measured set: z.x = z.x0 ^ g.u, g_a = z.G[a].
template <int MW>
__device__ inline void parity_form_wide(const uint64_t *md, uint32_t n_meas, const uint64_t *z, uint32_t &c,
                                        uint64_t (&g)[MW]) {
  uint32_t p = 0;
#pragma unroll
  for (int w = 0; w < MW; ++w) {
    p += __popcll(z[w] & md[w]);
    g[w] = 0;
  }
  c = p & 1u;
  for (uint32_t a = 0; a < n_meas; ++a) {
    const uint64_t *G = md + 2 * MW + (uint64_t)a * MW;
    uint32_t q = 0;
#pragma unroll
    for (int w = 0; w < MW; ++w) q += __popcll(z[w] & G[w]);
#pragma unroll
    for (int w = 0; w < MW; ++w)
      if ((a >> 6) == (uint32_t)w) g[w] |= (uint64_t)(q & 1u) << (a & 63);
  }
}

// Exact <(-1)^{z.x}>: (-1)^c if g = 0, else 0.  ext: [n_ext][MW].
template <int MW>
__global__ void parity_exact_wide_kernel(const uint64_t *__restrict__ models, uint32_t n_meas, uint64_t nv,
                                         const uint64_t *__restrict__ ext, uint32_t n_ext, double *__restrict__ E) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nv * n_ext) return;
  const uint64_t v = i / n_ext;
  const uint32_t s = (uint32_t)(i % n_ext);
  uint32_t c;
  uint64_t g[MW], any = 0;
  parity_form_wide<MW>(models + v * model_words(n_meas), n_meas, ext + (uint64_t)s * MW, c, g);
#pragma unroll
  for (int w = 0; w < MW; ++w) any |= g[w];
  E[i] = any ? 0.0 : (c ? -1.0 : 1.0);
}

// Odd-parity counts, bit-sliced as parity_sampled_kernel: lane l owns mask
// l of each group of 64, a wave draws 64 quads per round; for shot r the
// planes of the random bits in any form are ballots, a mask's parities
// over 64 shots the xor of the planes its form selects.  grid (nblk_x, nv).
template <int MW>
__global__ __launch_bounds__(kParityBlock) void parity_sampled_wide_kernel(
    const uint64_t *__restrict__ models, uint32_t n_meas, uint64_t shots, uint64_t seed, uint64_t vid0,
    const uint64_t *__restrict__ ext, uint32_t n_ext, uint32_t rounds, uint32_t *__restrict__ odd_counts) {
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t v = blockIdx.y;
  const uint64_t *md = models + v * model_words(n_meas);
  const uint64_t vid = vid0 + v;
  const uint64_t nquads = (shots + 3) >> 2;
  const uint64_t r0 = ((uint64_t)blockIdx.x * (kParityBlock / 64) + wave) * rounds;
  for (uint32_t p0 = 0; p0 < n_ext; p0 += 64) {
    const uint32_t s = p0 + lane;
    uint64_t g[MW], gall[MW];
    uint32_t cm = 0, cnt = 0;
#pragma unroll
    for (int w = 0; w < MW; ++w) g[w] = 0;
    if (s < n_ext) parity_form_wide<MW>(md, n_meas, ext + (uint64_t)s * MW, cm, g);
#pragma unroll
    for (int w = 0; w < MW; ++w) {
      uint64_t t = g[w];
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) t |= __shfl_xor(t, off);
      gall[w] = __builtin_amdgcn_readfirstlane((uint32_t)t) |
                ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(t >> 32)) << 32);
    }
    uint32_t total = 0;
    for (uint32_t rd = 0; rd < rounds; ++rd) {
      const uint64_t quad = (r0 + rd) * 64 + lane;
      uint64_t u[4][MW];
      if (quad < nquads) {
        quad_words<MW>(quad, vid, seed, n_meas, u);
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int w = 0; w < MW; ++w) u[r][w] = 0;
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint64_t valid = __ballot(quad < nquads && quad * 4 + r < shots);
        if (!valid) continue;
        total += __popcll(valid);
        uint64_t acc = 0;
#pragma unroll
        for (int w = 0; w < MW; ++w)
          for (uint64_t rem = gall[w]; rem; rem &= rem - 1) {
            const uint32_t j = (uint32_t)__builtin_ctzll(rem);
            const uint64_t plane = __ballot((u[r][w] >> j) & 1ull);
            acc ^= ((g[w] >> j) & 1ull) ? plane : 0ull;
          }
        cnt += __popcll(acc & valid);
      }
    }
    const uint32_t odd = cm ? total - cnt : cnt;
    if (s < n_ext && odd) atomicAdd(&odd_counts[v * n_ext + s], odd);
  }
}

// Shot records: records[v][shot][rw] (rw = ceil(n_meas / 64) words) =
// x0 ^ (xor of G[a] over the random a whose shot bit is set); one thread
// per shot, the model in LDS.
template <int MW>
__global__ __launch_bounds__(256) void records_wide_kernel(const uint64_t *__restrict__ models, uint32_t n_meas,
                                                           uint64_t shots, uint64_t seed, uint64_t vid0,
                                                           uint32_t rw, uint64_t *__restrict__ records) {
  extern __shared__ uint64_t s_md[];
  const uint64_t v = blockIdx.y;
  const uint32_t mw = model_words(n_meas);
  const uint64_t *md = models + v * mw;
  for (uint32_t i = threadIdx.x; i < mw; i += blockDim.x) s_md[i] = md[i];
  __syncthreads();
  const uint64_t shot = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (shot >= shots) return;
  uint64_t u[4][MW];
  quad_words<MW>(shot >> 2, vid0 + v, seed, n_meas, u);
  uint64_t x[MW], bits[MW];
#pragma unroll
  for (int w = 0; w < MW; ++w) {
    x[w] = s_md[w];
    bits[w] = s_md[MW + w];  // random measurements
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if ((shot & 3) == (uint64_t)r) bits[w] &= u[r][w];
  }
#pragma unroll
  for (int w = 0; w < MW; ++w)
    for (uint64_t rem = bits[w]; rem; rem &= rem - 1) {
      const uint32_t a = 64u * w + (uint32_t)__builtin_ctzll(rem);
      const uint64_t *G = s_md + 2 * MW + (uint64_t)a * MW;
#pragma unroll
      for (int k = 0; k < MW; ++k) x[k] ^= G[k];
    }
  uint64_t *dst = records + (v * shots + shot) * rw;
#pragma unroll
  for (int w = 0; w < MW; ++w)
    if ((uint32_t)w < rw) dst[w] = x[w];
}

}  // namespace

#define CCUT_MW_SWITCH(MW_, CALL) \
  switch (MW_) {                  \
    case 2: CALL(2); break;       \
    case 4: CALL(4); break;       \
    case 8: CALL(8); break;       \
    default: CALL(16); break;     \
  }

hipError_t launch_parity_exact_wide(const uint64_t *models, uint32_t n_meas, uint64_t nv, const uint64_t *ext,
                                    uint32_t n_ext, double *E, hipStream_t s) {
  if (n_meas <= (uint32_t)kMaxMeas || n_meas > (uint32_t)kMaxMeasWide) return hipErrorInvalidValue;
  const uint64_t n = nv * n_ext;
  if (n == 0) return hipSuccess;
  const dim3 g(blocks_for(n, 256)), b(256);
#define CCUT_PEW(M) hipLaunchKernelGGL(parity_exact_wide_kernel<M>, g, b, 0, s, models, n_meas, nv, ext, n_ext, E)
  CCUT_MW_SWITCH(model_mw(n_meas), CCUT_PEW)
#undef CCUT_PEW
  return hipGetLastError();
}

hipError_t launch_parity_sampled_wide(const uint64_t *models, uint32_t n_meas, uint64_t nv, uint64_t shots,
                                      uint64_t seed, uint64_t vid0, const uint64_t *ext, uint32_t n_ext,
                                      uint32_t *odd_counts, hipStream_t s) {
  if (n_meas <= (uint32_t)kMaxMeas || n_meas > (uint32_t)kMaxMeasWide || nv == 0 || nv > 65535)
    return hipErrorInvalidValue;
  if (shots == 0 || n_ext == 0) return hipSuccess;
  const uint64_t total_rounds = ((shots + 3) / 4 + 63) / 64;
  const uint64_t want_waves = std::max<uint64_t>(1, 4096 / nv);
  const uint64_t rounds = std::max<uint64_t>(1, (total_rounds + want_waves - 1) / want_waves);
  const uint64_t waves = (total_rounds + rounds - 1) / rounds;
  const uint64_t nbx = (waves + kParityBlock / 64 - 1) / (kParityBlock / 64);
  if (nbx > 0x7FFFFFFFull || rounds > 0xFFFFFFFFull) return hipErrorInvalidValue;
  const dim3 grid((unsigned)nbx, (unsigned)nv), block(kParityBlock);
#define CCUT_PSW(M)                                                                                            \
  hipLaunchKernelGGL(parity_sampled_wide_kernel<M>, grid, block, 0, s, models, n_meas, shots, seed, vid0, ext, \
                     n_ext, (uint32_t)rounds, odd_counts)
  CCUT_MW_SWITCH(model_mw(n_meas), CCUT_PSW)
#undef CCUT_PSW
  return hipGetLastError();
}

hipError_t launch_records_wide(const uint64_t *models, uint32_t n_meas, uint64_t nv, uint64_t shots, uint64_t seed,
                               uint64_t vid0, uint64_t *records, hipStream_t s) {
  if (n_meas <= (uint32_t)kMaxMeas || n_meas > (uint32_t)kMaxMeasWide || nv == 0 || nv > 65535)
    return hipErrorInvalidValue;
  if (shots == 0) return hipSuccess;
  const uint64_t nb = (shots + 255) / 256;
  if (nb > 0x7FFFFFFFull) return hipErrorInvalidValue;
  const size_t lds = (size_t)model_words(n_meas) * 8;
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  const dim3 grid((unsigned)nb, (unsigned)nv), block(256);
#define CCUT_RW(M)                                                                                         \
  do {                                                                                                     \
    hipError_t e = hipFuncSetAttribute((const void *)records_wide_kernel<M>,                               \
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);              \
    if (e != hipSuccess) return e;                                                                         \
    hipLaunchKernelGGL(records_wide_kernel<M>, grid, block, lds, s, models, n_meas, shots, seed, vid0,     \
                       (n_meas + 63) / 64, records);                                                      \
  } while (0)
  CCUT_MW_SWITCH(model_mw(n_meas), CCUT_RW)
#undef CCUT_RW
  return hipGetLastError();
}
#undef CCUT_MW_SWITCH

hipError_t launch_sample_hist(const uint64_t *models, uint32_t n_meas, uint64_t nv, uint64_t shots,
                              uint64_t seed, uint64_t vid0, uint32_t *partial, uint32_t nblk_x,
                              uint32_t qpt, uint64_t *records, hipStream_t s, const uint8_t *vmask) {
  if (n_meas > (uint32_t)kMaxMeas || nv == 0 || nv > 65535) return hipErrorInvalidValue;
  if (partial && n_meas <= kLdsHistBits && qpt > kMaxUnitQpt) return hipErrorInvalidValue;  // 16-bit LDS counts
  const size_t lds = sample_lds_bytes(n_meas, partial != nullptr);
  hipError_t e = hipFuncSetAttribute((const void *)sample_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sample_kernel, dim3(nblk_x, (unsigned)nv), dim3(kSampleBlock), lds, s, models,
                     n_meas, shots, seed, vid0, partial, qpt, records, vmask);
  return hipGetLastError();
}

hipError_t launch_sample_batch(const SampleJob *jobs, uint32_t n_jobs, uint64_t total_units, size_t lds,
                               hipStream_t s) {
  if (n_jobs == 0 || total_units == 0) return hipSuccess;
  if (lds > kSampleLdsMax) return hipErrorInvalidValue;
  // about 8192 workgroups, at most 8 units each
  const uint32_t per_wg = (uint32_t)std::min<uint64_t>(8, std::max<uint64_t>(1, total_units / 8192));
  const uint64_t wgs = (total_units + per_wg - 1) / per_wg;
  if (wgs > 0x7FFFFFFFull) return hipErrorInvalidValue;
  hipError_t e =
      hipFuncSetAttribute((const void *)sample_batch_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sample_batch_kernel, dim3((unsigned)wgs), dim3(kSampleBlock), lds, s, jobs, n_jobs, total_units,
                     per_wg);
  return hipGetLastError();
}

hipError_t launch_hist_reduce_batch(const SampleJob *jobs, uint32_t n_jobs, uint64_t total_reduce_blocks,
                                    hipStream_t s) {
  if (n_jobs == 0 || total_reduce_blocks == 0) return hipSuccess;
  if (total_reduce_blocks > 0x7FFFFFFFull) return hipErrorInvalidValue;
  hipLaunchKernelGGL(hist_reduce_batch_kernel, dim3((unsigned)total_reduce_blocks), dim3(256), 0, s, jobs, n_jobs);
  return hipGetLastError();
}

hipError_t launch_hist_reduce(const uint32_t *partial, uint64_t nv, uint32_t nblk, uint32_t bins,
                              uint64_t shots, double *dist, hipStream_t s, uint16_t *cnt16) {
  const uint64_t n = nv * bins;
  if (cnt16 && shots > 0xFFFFull) return hipErrorInvalidValue;
  hipLaunchKernelGGL(hist_reduce_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, partial, nv, nblk,
                     bins, shots, dist, cnt16);
  return hipGetLastError();
}

hipError_t launch_exact_tables(const uint64_t *models, uint32_t n_meas, uint64_t nv, double *dist,
                               hipStream_t s) {
  if (n_meas > (uint32_t)kMaxTableBits) return hipErrorInvalidValue;
  const uint64_t n = nv << n_meas;
  hipLaunchKernelGGL(exact_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, models, n_meas, nv, dist);
  return hipGetLastError();
}

hipError_t launch_parity_exact(const uint64_t *models, uint32_t n_meas, uint64_t nv,
                               const uint64_t *ext, uint32_t n_ext, double *E, hipStream_t s) {
  const uint64_t n = nv * n_ext;
  hipLaunchKernelGGL(parity_exact_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, models, n_meas, nv,
                     ext, n_ext, E);
  return hipGetLastError();
}

hipError_t launch_parity_sampled(const uint64_t *models, uint32_t n_meas, uint64_t nv, uint64_t shots,
                                 uint64_t seed, uint64_t vid0, const uint64_t *ext, uint32_t n_ext,
                                 uint32_t *odd_counts, hipStream_t s) {
  if (nv == 0 || nv > 65535) return hipErrorInvalidValue;
  if (shots == 0 || n_ext == 0) return hipSuccess;
  // rounds of 256 shots per wave: enough waves for about four per SIMD
  const uint64_t total_rounds = ((shots + 3) / 4 + 63) / 64;  // per variant
  const uint64_t want_waves = std::max<uint64_t>(1, 4096 / nv);
  const uint64_t rounds = std::max<uint64_t>(1, (total_rounds + want_waves - 1) / want_waves);
  const uint64_t waves = (total_rounds + rounds - 1) / rounds;
  const uint64_t nbx = (waves + kParityBlock / 64 - 1) / (kParityBlock / 64);
  if (nbx > 0x7FFFFFFFull || rounds > 0xFFFFFFFFull) return hipErrorInvalidValue;
  // per-workgroup sums in LDS while they fit in 64 KiB, else straight to memory
  const bool use_lds = n_ext <= 16384;
  const size_t lds = use_lds ? (size_t)n_ext * 4 : 0;
  const dim3 grid((unsigned)nbx, (unsigned)nv), block(kParityBlock);
  if (n_ext <= 64)
    hipLaunchKernelGGL(parity_sampled_kernel<1>, grid, block, lds, s, models, n_meas, shots, seed, vid0, ext, n_ext,
                       (uint32_t)rounds, (uint32_t)use_lds, odd_counts);
  else if (n_ext <= 128)
    hipLaunchKernelGGL(parity_sampled_kernel<2>, grid, block, lds, s, models, n_meas, shots, seed, vid0, ext, n_ext,
                       (uint32_t)rounds, (uint32_t)use_lds, odd_counts);
  else
    hipLaunchKernelGGL(parity_sampled_kernel<4>, grid, block, lds, s, models, n_meas, shots, seed, vid0, ext, n_ext,
                       (uint32_t)rounds, (uint32_t)use_lds, odd_counts);
  return hipGetLastError();
}

hipError_t launch_parity_finish(const uint32_t *odd, uint64_t n, uint64_t shots, bool settle, double *E,
                                hipStream_t s) {
  hipLaunchKernelGGL(parity_finish_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, odd, n, shots, settle ? 1 : 0,
                     E);
  return hipGetLastError();
}

hipError_t launch_dist_parity(const double *dist, uint32_t n_meas, uint64_t nv, const uint64_t *ext,
                              uint32_t n_ext, double *E, hipStream_t s) {
  if (n_meas > (uint32_t)kMaxNcQubits || nv == 0) return nv ? hipErrorInvalidValue : hipSuccess;
  const size_t lds = (size_t(1) << n_meas) * sizeof(double);
  for (uint64_t v0 = 0; v0 < nv; v0 += (1ull << 30)) {
    const uint64_t cnv = nv - v0 < (1ull << 30) ? nv - v0 : (1ull << 30);
    hipLaunchKernelGGL(dist_parity_kernel, dim3((unsigned)cnv), dim3(kWhtBlock), lds, s, dist + (v0 << n_meas),
                       n_meas, ext, n_ext, E + v0 * n_ext);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

namespace {
__global__ void fill_u32_kernel(uint32_t *p, uint64_t n, uint32_t value) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = value;
}
}  // namespace

hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t value, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<uint64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(fill_u32_kernel, dim3(blocks), dim3(256), 0, s, p, n, value);
  return hipGetLastError();
}

}  // namespace ccut

// Recombination as one dense contraction over the 4^k cut terms:
//   R[b] = 2^-k sum_P A[b_L; P] B[b_R; P],
//   A[b_L; P] = prod_{f in L} T_f[p_f(P)][b_f],  B[b_R; P] = prod_{f in R} T_f[p_f(P)][b_f],
// the tensor-network contraction of Sec. V-C grouped into two operands
// (one fragment on the column side, the rest on the row side).  Operand
// tiles are formed on the fly from the fragment tensors (never
// materialised: for 10 cuts the row operand alone would be 2^10 x 4^10).
//
// Precision modes:
//  - FP32 MFMA with FP64 across K tiles (the default fp32 mode): operands
//    rounded to fp32, one v_mfma_f32_16x16x4_f32 per 4 terms, products summed
//    in fp32 over 8 terms, those partial sums added into fp64 accumulators
//    (the signed sum over cut terms cancels heavily, so it is kept in fp64).
//    Each partial sum carries about 2^-23 relative error from the operand
//    rounding and the fp32 products and sums, so an output's error is about
//    2^-23 times the sum of its terms' magnitudes;
//  - the same with hi/lo split operands (a = a_hi + a_lo in fp32, three
//    MFMAs a_hi b_hi + a_hi b_lo + a_lo b_hi per 4 terms): the products are
//    then near fp64, but the fp32 sums over 8 terms still round at 2^-24
//    relative of the partial sum, so this gains a small constant factor at
//    three times the matrix-core work;
//  - FP64 MFMA (v_mfma_f64_16x16x4_f64) end to end (reference path).
// Split-K partials are summed in fp64 in split order by a second kernel.
// With a term list the K index runs over sampled terms P_j, each row-side
// value scaled by its importance weight (the estimator of the same sum);
// with `square` every operand value is squared first, which gives the sum
// of the squared sampled terms (the estimator's second moment).
#include <algorithm>

#include "common.hpp"

#pragma clang fp contract(off)

namespace ccut {

namespace {

constexpr int MT = 64, NT = 64, KC = 32, GEMM_THREADS = 256;

typedef float float4v __attribute__((ext_vector_type(4)));
typedef double double4v __attribute__((ext_vector_type(4)));

// The contraction's arguments as read-only (constant address space) data:
// read with a uniform index they compile to scalar loads, so operand
// formation keeps the descriptors out of the vector memory path.
typedef __attribute__((address_space(4))) const GemmArgs c_GemmArgs;
typedef __attribute__((address_space(4))) const RecombFrag c_RecombFrag;
__device__ inline c_GemmArgs *cargs(const GemmArgs *G) { return (c_GemmArgs *)(uint64_t)G; }

// p_f(P): the digits of P on fragment f's cuts
__device__ inline uint64_t frag_p(const GemmArgs *__restrict__ G, uint32_t f, uint64_t P) {
  c_GemmArgs *C = cargs(G);
  c_RecombFrag &F = C->f[f];
  if (C->ident[f]) return P;
  uint64_t p = 0;
  for (uint32_t j = 0; j < F.n_axes; ++j) p |= ((P >> (2 * F.axis_cut[j])) & 3ull) << (2 * j);
  return p;
}

// A fragment tensor entry: fp64, or a 16-bit shot count times fl(1/shots)
// (the value the fp64 table would hold).
__device__ inline double tval(const RecombFrag &F, uint64_t i) {
  return F.cnt16 ? (double)reinterpret_cast<const uint16_t *>(F.T)[i] * (1.0 / F.shots) : F.T[i];
}

__device__ inline double side_value(const GemmArgs *__restrict__ G, const GemmSide &S, uint32_t row, uint64_t P) {
  c_GemmArgs *C = cargs(G);
  const bool left = &S == &G->L;
  double v = 1.0;
  const uint32_t n = left ? C->L.n : C->R.n;
  for (uint32_t i = 0; i < n; ++i) {
    const uint32_t f = left ? C->L.frag[i] : C->R.frag[i];
    const uint32_t sh = left ? C->L.shift[i] : C->R.shift[i], bits = left ? C->L.bits[i] : C->R.bits[i];
    const uint32_t r = (row >> sh) & ((1u << bits) - 1u);
    c_RecombFrag &F = C->f[f];
    const uint64_t idx = frag_p(G, f, P) * F.rows + r;
    v *= F.cnt16 ? (double)reinterpret_cast<const uint16_t *>(F.T)[idx] * (1.0 / F.shots) : F.T[idx];
  }
  return v;
}

__device__ inline uint64_t out_index(const GemmArgs *__restrict__ G, uint32_t m, uint32_t n);
__device__ inline uint64_t side_bits(const GemmArgs *__restrict__ G, const GemmSide &S, uint32_t idx);

// A side that is one fragment whose axes are the cuts in order, with K
// running over every term: its operand is the fragment tensor itself
// (T[P][row], P-major), read with plain strided loads instead of
// side_value.  Returns the fragment, or null.
__device__ inline const RecombFrag *direct_side(const GemmArgs *__restrict__ G, const GemmSide &S) {
  c_GemmArgs *C = cargs(G);
  const bool left = &S == &G->L;
  const uint32_t n = left ? C->L.n : C->R.n;
  const uint32_t sh = left ? C->L.shift[0] : C->R.shift[0];
  if (n != 1 || C->terms || sh != 0) return nullptr;
  const uint32_t f = left ? C->L.frag[0] : C->R.frag[0];
  if (!C->ident[f]) return nullptr;
  return &G->f[f];
}

// A direct side's tensor as loop-invariant registers: read once through
// the constant address space (scalar loads), the entries through global
// pointers, so LDS stores of the operand tiles cannot be taken to alias
// them and no descriptor is reloaded per entry.
struct DirOp {
  const __attribute__((address_space(1))) double *T64;
  const __attribute__((address_space(1))) uint16_t *T16;
  double inv;  // fl(1 / shots): a count's value is count x inv
  uint64_t rows;
  bool c16;
};

__device__ inline DirOp dir_op(const RecombFrag *F) {
  DirOp D{};
  if (!F) return D;
  c_RecombFrag &C = *(c_RecombFrag *)(uint64_t)F;
  D.T64 = (const __attribute__((address_space(1))) double *)(uint64_t)C.T;
  D.T16 = (const __attribute__((address_space(1))) uint16_t *)(uint64_t)C.T;
  D.inv = 1.0 / C.shots;
  D.rows = C.rows;
  D.c16 = C.cnt16 != 0;
  return D;
}

// Entries (term kb + kk0 + STEP i, row col) of a direct side, i < NPER;
// 0 past the K range or the side's extent.  Every load is issued before
// the first is used (the value is tval's: count x fl(1/shots), or the fp64 entry).
template <uint32_t NPER, uint32_t STEP>
__device__ __attribute__((always_inline)) inline void direct_gather(const DirOp &D, uint64_t kb, uint64_t k1,
                                                                    uint32_t kk0, uint32_t col, bool col_ok,
                                                                    double *v) {
  uint64_t ix[NPER];
  bool ok[NPER];
#pragma unroll
  for (uint32_t i = 0; i < NPER; ++i) {
    const uint64_t j = kb + kk0 + STEP * i;
    ok[i] = col_ok && j < k1;
    ix[i] = ok[i] ? j * D.rows + col : 0;  // entry 0 stands in for the lanes past the range
  }
  if (D.c16) {
    uint32_t c[NPER];
#pragma unroll
    for (uint32_t i = 0; i < NPER; ++i) c[i] = D.T16[ix[i]];
#pragma unroll
    for (uint32_t i = 0; i < NPER; ++i) v[i] = ok[i] ? (double)c[i] * D.inv : 0.0;
  } else {
#pragma unroll
    for (uint32_t i = 0; i < NPER; ++i) v[i] = D.T64[ix[i]];
#pragma unroll
    for (uint32_t i = 0; i < NPER; ++i) v[i] = ok[i] ? v[i] : 0.0;
  }
}

// direct_gather in two steps, so a chunk's loads can be issued a chunk
// ahead: the raw entries (16-bit count or fp64 bits) ...
template <uint32_t NPER, uint32_t STEP>
__device__ __attribute__((always_inline)) inline void direct_load(const DirOp &D, uint64_t kb, uint64_t k1,
                                                                  uint32_t kk0, uint32_t col, bool col_ok,
                                                                  uint64_t *raw) {
  uint64_t ix[NPER];
#pragma unroll
  for (uint32_t i = 0; i < NPER; ++i) {
    const uint64_t j = kb + kk0 + STEP * i;
    ix[i] = col_ok && j < k1 ? j * D.rows + col : 0;
  }
  if (D.c16) {
#pragma unroll
    for (uint32_t i = 0; i < NPER; ++i) raw[i] = D.T16[ix[i]];
  } else {
#pragma unroll
    for (uint32_t i = 0; i < NPER; ++i) raw[i] = (uint64_t)__double_as_longlong(D.T64[ix[i]]);
  }
}
// ... and their values (0 past the K range or the side's extent)
template <uint32_t NPER, uint32_t STEP>
__device__ __attribute__((always_inline)) inline void direct_value(const DirOp &D, uint64_t kb, uint64_t k1,
                                                                   uint32_t kk0, bool col_ok, const uint64_t *raw,
                                                                   double *v) {
#pragma unroll
  for (uint32_t i = 0; i < NPER; ++i) {
    const bool ok = col_ok && kb + kk0 + STEP * i < k1;
    const double x = D.c16 ? (double)(uint32_t)raw[i] * D.inv : __longlong_as_double((long long)raw[i]);
    v[i] = ok ? x : 0.0;
  }
}

// Operand factors of a side that is not one direct fragment: the tile's
// 64 rows (or columns) take only 2^vb distinct row values of fragment t
// (vb = its row bits below bit 6 of the side index; the 64 indices share
// every higher bit), so per K chunk fragment t's factors
// F_t[kk][r] = T_t[p_t(P_kk)][fixed_t | r] are gathered once into LDS and
// each operand entry is their product in fragment order (the product
// side_value forms, the same roundings).  Layout per side: fragment t at
// word offset KC (cnt_0 + ... + cnt_{t-1}), [kk][r].  At most kFacFrags
// fragments per side (more: side_value per entry).
constexpr uint32_t kFacFrags = 8;

__host__ __device__ inline uint32_t fac_vb(uint32_t shift, uint32_t bits) {
  return shift >= 6 ? 0u : (bits < 6 - shift ? bits : 6 - shift);
}

// Doubles of LDS the factor tables of side S take (0: no tables).
__host__ __device__ inline uint32_t fac_words(const GemmArgs &h, const GemmSide &S) {
  if (S.n > kFacFrags || (S.n == 1 && !h.terms && S.shift[0] == 0 && h.ident[S.frag[0]])) return 0;
  uint32_t w = 0;
  for (uint32_t t = 0; t < S.n; ++t) w += KC << fac_vb(S.shift[t], S.bits[t]);
  return w;
}

// Fill side S's factor tables for the tile whose first index is base:
// fragment by fragment (uniform), one gather per entry.
__device__ inline void fac_fill(const GemmArgs *__restrict__ G, bool left, uint32_t base, uint64_t kb, uint64_t k1,
                                double *__restrict__ fac) {
  c_GemmArgs *C = cargs(G);
  const uint32_t n = left ? C->L.n : C->R.n;
  uint32_t off = 0;
  for (uint32_t t = 0; t < n; ++t) {
    const uint32_t f = left ? C->L.frag[t] : C->R.frag[t];
    const uint32_t sh = left ? C->L.shift[t] : C->R.shift[t], bits = left ? C->L.bits[t] : C->R.bits[t];
    const uint32_t vb = fac_vb(sh, bits), cnt = 1u << vb;
    const uint32_t fixed = (base >> sh) & ((1u << bits) - 1u);
    c_RecombFrag &F = C->f[f];
    for (uint32_t e = threadIdx.x; e < KC * cnt; e += GEMM_THREADS) {
      const uint32_t kk = e >> vb, r = e & (cnt - 1u);
      const uint64_t j = kb + kk;
      double v = 0.0;
      if (j < k1) {
        const uint64_t idx = frag_p(G, f, C->terms ? C->terms[j] : j) * F.rows + (fixed | r);
        v = F.cnt16 ? (double)reinterpret_cast<const uint16_t *>(F.T)[idx] * (1.0 / F.shots) : F.T[idx];
      }
      fac[off + e] = v;
    }
    off += KC * cnt;
  }
}

// Entry (kk, local) of a factored side: the product of its fragments'
// factors in fragment order.
__device__ inline double fac_value(const GemmArgs *__restrict__ G, bool left, const double *__restrict__ fac,
                                   uint32_t kk, uint32_t local) {
  c_GemmArgs *C = cargs(G);
  const uint32_t n = left ? C->L.n : C->R.n;
  double v = 1.0;
  uint32_t off = 0;
  for (uint32_t t = 0; t < n; ++t) {
    const uint32_t sh = left ? C->L.shift[t] : C->R.shift[t], bits = left ? C->L.bits[t] : C->R.bits[t];
    const uint32_t vb = fac_vb(sh, bits);
    v *= fac[off + (kk << vb) + ((local >> sh) & ((1u << vb) - 1u))];
    off += KC << vb;
  }
  return v;
}

// One 64 x 64 output tile (tile index `tile`, M tiles fastest) over the
// K range of split `split`, into partial[split][M][N].  MODE 0: fp64
// MFMA; 1: fp32 operands, one fp32 MFMA product per term; 2: hi/lo split
// fp32 operands, three products.  GEN false: both sides are one fragment
// read directly (direct_side); true: any side, a side that is not direct
// formed from factor tables (dynamic LDS: the row side's, then the column
// side's, fac_words each) or, beyond kFacFrags fragments, per entry.
template <int MODE, bool GEN>
__device__ __attribute__((always_inline)) inline void gemm_body(const GemmArgs *__restrict__ G, uint64_t k_per_split,
                                                               double *__restrict__ partial,
                                 uint32_t tile, uint32_t split, double *__restrict__ out = nullptr) {
  constexpr bool F32 = MODE != 0, LO = MODE == 2;
  typedef typename std::conditional<F32, float, double>::type TS;
  __shared__ TS As[KC][MT + 1];
  __shared__ TS Bs[KC][NT + 1];
  __shared__ TS Al[LO ? KC : 1][MT + 1];  // hi/lo mode: low parts of the split operands
  __shared__ TS Bl[LO ? KC : 1][NT + 1];
  const uint32_t M = G->M, N = G->N;
  const uint64_t K = G->K;
  const uint32_t tilesM = (M + MT - 1) / MT;
  const uint32_t tm = tile % tilesM, tn = tile / tilesM;
  const uint64_t k0 = (uint64_t)split * k_per_split;
  const uint64_t k1 = std::min<uint64_t>(K, k0 + k_per_split);
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  double acc64[2][2][4];
  float4v acc32[2][2];
  double4v accd[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      acc32[i][j] = float4v{0.f, 0.f, 0.f, 0.f};
      accd[i][j] = double4v{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int g = 0; g < 4; ++g) acc64[i][j][g] = 0.0;
    }
  const RecombFrag *FA = direct_side(G, G->L), *FB = direct_side(G, G->R);
  const DirOp DA = dir_op(FA), DB = dir_op(FB);
  extern __shared__ double s_fac[];
  uint32_t wA = 0, wB = 0;
  if constexpr (GEN) {
    wA = fac_words(*G, G->L);
    wB = fac_words(*G, G->R);
  }
  double *facA = s_fac, *facB = s_fac + wA;
  // the arguments read once (uniform), not per operand entry
  const double *tscale = G->tscale;
  const __attribute__((address_space(1))) double *tscale_g = (const __attribute__((address_space(1))) double *)tscale;
  const uint64_t *terms = G->terms;
  const bool square = G->square != 0;
  // output index bits of the tile's rows and columns (written with the
  // outputs directly when there is one split)
  __shared__ uint64_t s_obits[MT + NT];
  if (out) {
    if (tid < MT) s_obits[tid] = tm * MT + tid < M ? side_bits(G, G->L, tm * MT + tid) : 0;
    else if (tid < MT + NT) s_obits[tid] = tn * NT + tid - MT < N ? side_bits(G, G->R, tn * NT + tid - MT) : 0;
    __syncthreads();
  }
  // both sides direct (GEN false): the next chunk's raw entries are loaded
  // into registers while this chunk's products run
  constexpr uint32_t NPA = KC * MT / GEMM_THREADS, STA = GEMM_THREADS / MT;
  constexpr uint32_t NPB = KC * NT / GEMM_THREADS, STB = GEMM_THREADS / NT;
  const uint32_t mmA = tid % MT, kkA = tid / MT, mA = tm * MT + mmA;
  const uint32_t nnB = tid % NT, kkB = tid / NT, nB = tn * NT + nnB;
  uint64_t rawA[GEN ? 1 : NPA], rawB[GEN ? 1 : NPB];
  auto prefetch = [&](uint64_t kb) {
    if constexpr (!GEN) {
      direct_load<NPA, STA>(DA, kb, k1, kkA, mA, mA < M, rawA);
      direct_load<NPB, STB>(DB, kb, k1, kkB, nB, nB < N, rawB);
    }
  };
  prefetch(k0);
  for (uint64_t kb = k0; kb < k1; kb += KC) {
    if constexpr (!GEN) {
      double a[NPA], b[NPB];
      direct_value<NPA, STA>(DA, kb, k1, kkA, mA < M, rawA, a);
      direct_value<NPB, STB>(DB, kb, k1, kkB, nB < N, rawB, b);
#pragma unroll
      for (uint32_t i = 0; i < NPA; ++i) {
        double x = a[i];
        const uint64_t j = kb + kkA + STA * i;
        if (tscale && mA < M && j < k1) x *= tscale_g[j];  // (term weights: not prefetched, rarely set here)
        if (square) x *= x;
        As[kkA + STA * i][mmA] = (TS)x;
        if constexpr (LO) Al[kkA + STA * i][mmA] = (float)(x - (double)(float)x);
      }
#pragma unroll
      for (uint32_t i = 0; i < NPB; ++i) {
        double x = b[i];
        if (square) x *= x;
        Bs[kkB + STB * i][nnB] = (TS)x;
        if constexpr (LO) Bl[kkB + STB * i][nnB] = (float)(x - (double)(float)x);
      }
    } else {
      if constexpr (GEN) {
        if (wA || wB) {
          if (wA) fac_fill(G, true, tm * MT, kb, k1, facA);
          if (wB) fac_fill(G, false, tn * NT, kb, k1, facB);
          __syncthreads();
        }
      }
      if (!GEN || FA) {
        // one fragment read directly: a thread's entries share its row
        constexpr uint32_t NPA = KC * MT / GEMM_THREADS, STA = GEMM_THREADS / MT;
        const uint32_t mm = tid % MT, kk0 = tid / MT, m = tm * MT + mm;
        double a[NPA];
        direct_gather<NPA, STA>(DA, kb, k1, kk0, m, m < M, a);
        double ts[NPA];
#pragma unroll
        for (uint32_t i = 0; i < NPA; ++i) {
          const uint64_t j = kb + kk0 + STA * i;
          ts[i] = (tscale && m < M && j < k1) ? tscale_g[j] : 1.0;
        }
#pragma unroll
        for (uint32_t i = 0; i < NPA; ++i) {
          double x = a[i];
          if (tscale) x *= ts[i];
          if (square) x *= x;
          As[kk0 + STA * i][mm] = (TS)x;
          if constexpr (LO) Al[kk0 + STA * i][mm] = (float)(x - (double)(float)x);
        }
      } else {
        for (uint32_t e = tid; e < KC * MT; e += GEMM_THREADS) {
          const uint32_t kk = e / MT, mm = e % MT;
          const uint32_t m = tm * MT + mm;
          const uint64_t j = kb + kk;
          double a = 0.0;
          if (m < M && j < k1) {
            a = wA ? fac_value(G, true, facA, kk, mm) : side_value(G, G->L, m, terms ? terms[j] : j);
            if (tscale) a *= tscale[j];
            if (square) a *= a;
          }
          As[kk][mm] = (TS)a;
          if constexpr (LO) Al[kk][mm] = (float)(a - (double)(float)a);
        }
      }
      if (!GEN || FB) {
        constexpr uint32_t NPB = KC * NT / GEMM_THREADS, STB = GEMM_THREADS / NT;
        const uint32_t nn = tid % NT, kk0 = tid / NT, n = tn * NT + nn;
        double b[NPB];
        direct_gather<NPB, STB>(DB, kb, k1, kk0, n, n < N, b);
#pragma unroll
        for (uint32_t i = 0; i < NPB; ++i) {
          double x = b[i];
          if (square) x *= x;
          Bs[kk0 + STB * i][nn] = (TS)x;
          if constexpr (LO) Bl[kk0 + STB * i][nn] = (float)(x - (double)(float)x);
        }
      } else {
        for (uint32_t e = tid; e < KC * NT; e += GEMM_THREADS) {
          const uint32_t kk = e / NT, nn = e % NT;
          const uint32_t n = tn * NT + nn;
          const uint64_t j = kb + kk;
          double b = 0.0;
          if (n < N && j < k1) b = wB ? fac_value(G, false, facB, kk, nn) : side_value(G, G->R, n, terms ? terms[j] : j);
          if (square) b *= b;
          Bs[kk][nn] = (TS)b;
          if constexpr (LO) Bl[kk][nn] = (float)(b - (double)(float)b);
        }
      }
    }
    __syncthreads();
    if (kb + KC < k1) prefetch(kb + KC);  // in flight during the products below
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      TS a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[kk + lane / 16][wm + 16 * i + lane % 16];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[kk + lane / 16][wn + 16 * j + lane % 16];
      if constexpr (F32) {
        if constexpr (LO) {
          float al[2], bl[2];
#pragma unroll
          for (int i = 0; i < 2; ++i) al[i] = Al[kk + lane / 16][wm + 16 * i + lane % 16];
#pragma unroll
          for (int j = 0; j < 2; ++j) bl[j] = Bl[kk + lane / 16][wn + 16 * j + lane % 16];
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
              acc32[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32((float)a[i], bl[j], acc32[i][j], 0, 0, 0);
              acc32[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(al[i], (float)b[j], acc32[i][j], 0, 0, 0);
            }
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc32[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32((float)a[i], (float)b[j], acc32[i][j], 0, 0, 0);
        if (kk & 4) {  // fold every 8 terms into fp64
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
#pragma unroll
              for (int g = 0; g < 4; ++g) acc64[i][j][g] += (double)acc32[i][j][g];
              acc32[i][j] = float4v{0.f, 0.f, 0.f, 0.f};
            }
        }
      } else {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            accd[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)a[i], (double)b[j], accd[i][j], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  double *dst = partial + (uint64_t)split * M * N;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        // accumulator register g of a lane holds row 4 (lane / 16) + g of the
        // 16x16 block for the fp32 instruction, row lane / 16 + 4 g for fp64
        const uint32_t r = F32 ? 4 * (lane / 16) + g : lane / 16 + 4 * g;
        const uint32_t m = tm * MT + wm + 16 * i + r;
        const uint32_t n = tn * NT + wn + 16 * j + lane % 16;
        if (m >= M || n >= N) continue;
        const double v = F32 ? acc64[i][j][g] : accd[i][j][g];
        // one split: the output itself (as the reduction would write it)
        if (out) out[s_obits[m - tm * MT] | s_obits[MT + n - tn * NT]] = ldexp(0.0 + v, -(int)G->k);
        else dst[(uint64_t)m * N + n] = v;
      }
}

template <int MODE, bool GEN>
__global__ __launch_bounds__(GEMM_THREADS, 3) void gemm_kernel(const GemmArgs *__restrict__ G, uint64_t k_per_split,
                                                            double *__restrict__ partial, double *__restrict__ out) {
  gemm_body<MODE, GEN>(G, k_per_split, partial, blockIdx.x, blockIdx.y, out);
}

// Many contractions in one launch: workgroup x runs tile (x - wg0) mod
// tiles, split (x - wg0) / tiles of the job holding x.
template <int MODE, bool GEN>
__global__ __launch_bounds__(GEMM_THREADS, 3) void gemm_batch_kernel(const GemmJob *__restrict__ jobs, uint32_t n_jobs) {
  const uint32_t bid = xcd_block(blockIdx.x, gridDim.x);  // the tiles of a job share one XCD's L2
  const uint32_t j = find_job(jobs, n_jobs, bid, [](const GemmJob &J) { return J.wg0; });
  const GemmJob &J = jobs[j];
  const uint64_t local = bid - J.wg0;
  gemm_body<MODE, GEN>(J.args, J.k_per_split, J.partial, (uint32_t)(local % J.tiles), (uint32_t)(local / J.tiles),
                       J.splits == 1 ? *J.out : nullptr);
}

// Skinny contraction (M <= SK_M rows, fp64): CPT adjacent output columns
// per thread with all M rows in registers; the row-side values of a K chunk
// are staged in LDS.  partial[split][m][n] = sum over the split's terms, in
// ascending order, of a(m, P) * b(n, P) (each product rounded, then added).
// A thread's CPT columns come in one vector load per term (CPT 16-bit shot
// counts in 8 bytes, or CPT doubles), so a wave moves 512 bytes or more per
// load instruction.
constexpr uint32_t SK_N = 256, SK_M = 32, SK_KC = 64;

// Column loads through global pointers: vector-memory loads only, so the
// LDS reads of the loop never wait for them.
typedef const __attribute__((address_space(1))) uint16_t g_u16;
typedef const __attribute__((address_space(1))) double g_f64;
typedef double d2v __attribute__((ext_vector_type(2)));
typedef uint32_t u2v __attribute__((ext_vector_type(2)));

template <uint32_t CPT>
struct ColLoad;
template <>
struct ColLoad<1> {
  typedef uint32_t Raw16;
  typedef double Raw64;
  __device__ static Raw16 cnt(g_u16 *p) { return p[0]; }
  __device__ static void cnt_val(Raw16 w, double inv, double *b) { b[0] = (double)w * inv; }
  __device__ static Raw64 f64(g_f64 *p) { return p[0]; }
  __device__ static void f64_val(Raw64 v, double *b) { b[0] = v; }
};
template <>
struct ColLoad<2> {
  typedef uint32_t Raw16;
  typedef d2v Raw64;
  __device__ static Raw16 cnt(g_u16 *p) { return *reinterpret_cast<const __attribute__((address_space(1))) uint32_t *>(p); }
  __device__ static void cnt_val(Raw16 w, double inv, double *b) {
    b[0] = (double)(w & 0xFFFFu) * inv;
    b[1] = (double)(w >> 16) * inv;
  }
  __device__ static Raw64 f64(g_f64 *p) { return *reinterpret_cast<const __attribute__((address_space(1))) d2v *>(p); }
  __device__ static void f64_val(Raw64 v, double *b) { b[0] = v.x, b[1] = v.y; }
};
template <>
struct ColLoad<4> {
  typedef u2v Raw16;
  struct Raw64 {
    d2v a, b;
  };
  __device__ static Raw16 cnt(g_u16 *p) { return *reinterpret_cast<const __attribute__((address_space(1))) u2v *>(p); }
  __device__ static void cnt_val(Raw16 w, double inv, double *b) {
    b[0] = (double)(w.x & 0xFFFFu) * inv;
    b[1] = (double)(w.x >> 16) * inv;
    b[2] = (double)(w.y & 0xFFFFu) * inv;
    b[3] = (double)(w.y >> 16) * inv;
  }
  __device__ static Raw64 f64(g_f64 *p) {
    const __attribute__((address_space(1))) d2v *q = reinterpret_cast<const __attribute__((address_space(1))) d2v *>(p);
    return Raw64{q[0], q[1]};
  }
  __device__ static void f64_val(Raw64 v, double *b) { b[0] = v.a.x, b[1] = v.a.y, b[2] = v.b.x, b[3] = v.b.y; }
};

// One instantiation per row count MC (1, 2, ..., 32) and column count CPT:
// the accumulators of one kernel stay in registers only when the kernel
// holds exactly its own.
template <uint32_t MC, uint32_t CPT>
__device__ __attribute__((always_inline)) inline void skinny_body(const GemmArgs *__restrict__ G, uint64_t k_per_split, double *__restrict__ partial,
                                   uint32_t tile, uint32_t split, double *__restrict__ out) {
  __shared__ double As[SK_KC][MC];
  __shared__ uint64_t s_boff[SK_KC];
  const uint32_t N = G->N, tid = threadIdx.x;
  const uint64_t K = G->K;
  const uint32_t n = (tile * SK_N + tid) * CPT;  // the thread's first column (N is a multiple of CPT)
  const uint64_t k0 = (uint64_t)split * k_per_split;
  const uint64_t k1 = std::min<uint64_t>(K, k0 + k_per_split);
  // the column side is one fragment whose rows are the column index
  const uint32_t rf = G->R.frag[0];
  c_RecombFrag &FR = cargs(G)->f[rf];
  g_f64 *Tn = (g_f64 *)(uint64_t)FR.T + n;
  g_u16 *Cn = (g_u16 *)(uint64_t)FR.T + n;
  const bool cnt16 = FR.cnt16 != 0;
  const double inv = 1.0 / FR.shots;  // a count's value is count x fl(1/shots)
  const uint64_t rows = FR.rows;
  const bool square = G->square != 0;
  g_f64 *tscale = (g_f64 *)(uint64_t)cargs(G)->tscale;
  const uint64_t *terms = cargs(G)->terms;
  const RecombFrag *FA = direct_side(G, G->L);
  const DirOp DA = dir_op(FA);
  __shared__ uint64_t s_mbits[MC];  // output index bits of the rows
  if (out) {
    if (tid < MC) s_mbits[tid] = side_bits(G, G->L, tid);
    __syncthreads();
  }
  double acc[MC][CPT];
#pragma unroll
  for (uint32_t m = 0; m < MC; ++m)
#pragma unroll
    for (uint32_t c = 0; c < CPT; ++c) acc[m][c] = 0.0;
  for (uint64_t kb = k0; kb < k1; kb += SK_KC) {
    const uint32_t kn = (uint32_t)std::min<uint64_t>(SK_KC, k1 - kb);
    __syncthreads();  // the previous chunk is consumed
    if (tid < kn) {
      const uint64_t j = kb + tid;
      s_boff[tid] = frag_p(G, rf, terms ? terms[j] : j) * rows;
    }
    for (uint32_t e = tid; e < kn * MC; e += SK_N) {
      const uint32_t kk = e / MC, m = e % MC;
      const uint64_t j = kb + kk;
      double a;
      if (FA) {
        const uint64_t ix = j * DA.rows + m;
        a = DA.c16 ? (double)DA.T16[ix] * DA.inv : DA.T64[ix];
      } else {
        a = side_value(G, G->L, m, terms ? terms[j] : j);
      }
      if (tscale) a *= tscale[j];
      if (square) a *= a;
      As[kk][m] = a;
    }
    __syncthreads();
    if (n >= N) continue;
    // the column tensor streamed once: a batch of U terms' loads issued
    // before the first is used (fewer for many accumulators, which would
    // crowd the registers)
    constexpr uint32_t U = MC * CPT <= 8 ? 8 : 4;
    if (cnt16) {  // 16-bit shot counts: a quarter of the bytes, the same values
      for (uint32_t k2 = 0; k2 < kn; k2 += U) {
        typename ColLoad<CPT>::Raw16 w[U];
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) w[u] = ColLoad<CPT>::cnt(Cn + s_boff[k2 + u < kn ? k2 + u : k2]);
        __builtin_amdgcn_sched_barrier(0);  // the loads stay ahead of their uses
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
          if (k2 + u >= kn) break;
          double b[CPT];
          ColLoad<CPT>::cnt_val(w[u], inv, b);
#pragma unroll
          for (uint32_t c = 0; c < CPT; ++c) {
            if (square) b[c] *= b[c];
#pragma unroll
            for (uint32_t m = 0; m < MC; ++m) acc[m][c] += As[k2 + u][m] * b[c];
          }
        }
      }
    } else {
      for (uint32_t k2 = 0; k2 < kn; k2 += U) {
        typename ColLoad<CPT>::Raw64 w[U];
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) w[u] = ColLoad<CPT>::f64(Tn + s_boff[k2 + u < kn ? k2 + u : k2]);
        __builtin_amdgcn_sched_barrier(0);  // the loads stay ahead of their uses
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
          if (k2 + u >= kn) break;
          double b[CPT];
          ColLoad<CPT>::f64_val(w[u], b);
#pragma unroll
          for (uint32_t c = 0; c < CPT; ++c) {
            if (square) b[c] *= b[c];
#pragma unroll
            for (uint32_t m = 0; m < MC; ++m) acc[m][c] += As[k2 + u][m] * b[c];
          }
        }
      }
    }
  }
  if (n >= N) return;
  if (out) {
#pragma unroll
    for (uint32_t c = 0; c < CPT; ++c) {
      const uint64_t nb = side_bits(G, G->R, n + c);
#pragma unroll
      for (uint32_t m = 0; m < MC; ++m) out[s_mbits[m] | nb] = ldexp(0.0 + acc[m][c], -(int)G->k);
    }
    return;
  }
  double *dst = partial + (uint64_t)split * MC * N;
#pragma unroll
  for (uint32_t m = 0; m < MC; ++m)
#pragma unroll
    for (uint32_t c = 0; c < CPT; ++c) dst[(uint64_t)m * N + n + c] = acc[m][c];
}

template <uint32_t MC, uint32_t CPT>
__global__ __launch_bounds__(SK_N) void skinny_kernel(const GemmArgs *__restrict__ G, uint64_t k_per_split,
                                                      double *__restrict__ partial, double *__restrict__ out) {
  skinny_body<MC, CPT>(G, k_per_split, partial, blockIdx.x, blockIdx.y, out);
}

// Jobs of one row count MC and column count CPT.
template <uint32_t MC, uint32_t CPT>
__global__ __launch_bounds__(SK_N) void skinny_batch_kernel(const GemmJob *__restrict__ jobs, uint32_t n_jobs) {
  const uint32_t j = find_job(jobs, n_jobs, blockIdx.x, [](const GemmJob &J) { return J.wg0; });
  const GemmJob &J = jobs[j];
  const uint64_t local = blockIdx.x - J.wg0;
  skinny_body<MC, CPT>(J.args, J.k_per_split, J.partial, (uint32_t)(local % J.tiles), (uint32_t)(local / J.tiles),
                       J.splits == 1 ? *J.out : nullptr);
}

// The skinny kernel for M rows and CPT columns per thread, one launch.
// batch: the job list (grid total_wg), else one contraction (grid tiles x splits).
template <uint32_t MC, uint32_t CPT>
void skinny_launch(dim3 g, hipStream_t s, const GemmJob *jobs, uint32_t n_jobs, const GemmArgs *args,
                   uint64_t k_per_split, double *partial, double *out) {
  if (jobs)
    hipLaunchKernelGGL((skinny_batch_kernel<MC, CPT>), g, dim3(SK_N), 0, s, jobs, n_jobs);
  else
    hipLaunchKernelGGL((skinny_kernel<MC, CPT>), g, dim3(SK_N), 0, s, args, k_per_split, partial, out);
}

template <uint32_t MC>
hipError_t skinny_cols_launch(uint32_t cpt, dim3 g, hipStream_t s, const GemmJob *jobs, uint32_t n_jobs,
                              const GemmArgs *args, uint64_t k_per_split, double *partial, double *out) {
  switch (cpt) {
    case 1: skinny_launch<MC, 1>(g, s, jobs, n_jobs, args, k_per_split, partial, out); break;
    case 2: skinny_launch<MC, 2>(g, s, jobs, n_jobs, args, k_per_split, partial, out); break;
    case 4:
      if constexpr (MC <= 4) {
        skinny_launch<MC, 4>(g, s, jobs, n_jobs, args, k_per_split, partial, out);
        break;
      }
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t skinny_dispatch(uint32_t rows, uint32_t cpt, dim3 g, hipStream_t s, const GemmJob *jobs, uint32_t n_jobs,
                           const GemmArgs *args, uint64_t k_per_split, double *partial, double *out) {
  switch (rows) {
    case 1: return skinny_cols_launch<1>(cpt, g, s, jobs, n_jobs, args, k_per_split, partial, out);
    case 2: return skinny_cols_launch<2>(cpt, g, s, jobs, n_jobs, args, k_per_split, partial, out);
    case 4: return skinny_cols_launch<4>(cpt, g, s, jobs, n_jobs, args, k_per_split, partial, out);
    case 8: return skinny_cols_launch<8>(cpt, g, s, jobs, n_jobs, args, k_per_split, partial, out);
    case 16: return skinny_cols_launch<16>(cpt, g, s, jobs, n_jobs, args, k_per_split, partial, out);
    case 32: return cpt == 1 ? skinny_cols_launch<32>(cpt, g, s, jobs, n_jobs, args, k_per_split, partial, out)
                             : hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

// The output index bits of row (or column) idx of side S: each of its
// fragments' requested bits at its user position.
__device__ inline uint64_t side_bits(const GemmArgs *__restrict__ G, const GemmSide &S, uint32_t idx) {
  // the descriptors are uniform: scalar loads through the constant space
  c_GemmArgs *C = cargs(G);
  const bool left = &S == &G->L;
  const uint32_t n = left ? C->L.n : C->R.n;
  uint64_t b = 0;
  for (uint32_t t = 0; t < n; ++t) {
    const uint32_t f = left ? C->L.frag[t] : C->R.frag[t];
    const uint32_t sh = left ? C->L.shift[t] : C->R.shift[t], bits = left ? C->L.bits[t] : C->R.bits[t];
    c_RecombFrag &F = C->f[f];
    const uint32_t r = (idx >> sh) & ((1u << bits) - 1u);
    for (uint32_t q = 0; q < F.n_req; ++q) b |= (uint64_t)((r >> q) & 1u) << F.req_user[q];
  }
  return b;
}

// out[b(m, n)] = 2^-k sum_split partial[split][m][n], splits in order
__device__ inline uint64_t out_index(const GemmArgs *__restrict__ G, uint32_t m, uint32_t n) {
  return side_bits(G, G->L, m) | side_bits(G, G->R, n);
}

__device__ inline void gemm_reduce_body(const GemmArgs *__restrict__ G, const double *__restrict__ partial,
                                        uint32_t splits, double *__restrict__ out, uint64_t i) {
  const uint64_t MN = (uint64_t)G->M * G->N;
  if (i >= MN) return;
  double s = 0.0;
  for (uint32_t sp = 0; sp < splits; ++sp) s += partial[sp * MN + i];
  out[out_index(G, (uint32_t)(i / G->N), (uint32_t)(i % G->N))] = ldexp(s, -(int)G->k);
}

__global__ void gemm_reduce_kernel(const GemmArgs *__restrict__ G, const double *__restrict__ partial,
                                   uint32_t splits, double *__restrict__ out) {
  gemm_reduce_body(G, partial, splits, out, (uint64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ void gemm_reduce_batch_kernel(const GemmJob *__restrict__ jobs, uint32_t n_jobs) {
  const uint32_t j = find_job(jobs, n_jobs, blockIdx.x, [](const GemmJob &J) { return J.rwg0; });
  const GemmJob &J = jobs[j];
  gemm_reduce_body(J.args, J.partial, J.splits, *J.out, (blockIdx.x - J.rwg0) * 256ull + threadIdx.x);
}

}  // namespace

// K splits: about 1024 workgroups, each split at least 8 K chunks (256
// terms), so short contractions take one split and write their outputs
// directly (no partial sums, no reduction pass).
uint32_t gemm_splits(const GemmArgs &h) {
  const uint64_t tiles = (uint64_t)((h.M + MT - 1) / MT) * ((h.N + NT - 1) / NT);
  const uint64_t kchunks = (h.K + KC - 1) / KC;
  uint64_t s = std::max<uint64_t>(1, 1024 / std::max<uint64_t>(tiles, 1));
  s = std::min<uint64_t>(s, kchunks / 8);
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(s, 65535));
}

// rows a power of two up to 32 (the row side's requested bits), one column fragment
bool contraction_skinny(const GemmArgs &h, bool fp32) {
  return !fp32 && h.M <= SK_M && (h.M & (h.M - 1)) == 0 && h.R.n == 1 && h.R.shift[0] == 0;
}

// Columns per thread of the skinny kernel: 4 for at most 4 rows, 2 for 8
// and 16, 1 for 32 (at most 32 accumulators), and never more than N (a
// power of two: the rows of the one column fragment).
uint32_t skinny_cols(const GemmArgs &h) {
  const uint32_t cap = h.M <= 4 ? 4 : h.M <= 16 ? 2 : 1;
  return std::min<uint32_t>(cap, h.N);
}

uint32_t gemm_tiles(const GemmArgs &h, bool skinny) {
  if (skinny) return (h.N + SK_N * skinny_cols(h) - 1) / (SK_N * skinny_cols(h));
  return ((h.M + MT - 1) / MT) * ((h.N + NT - 1) / NT);
}

uint32_t contraction_splits(const GemmArgs &h, bool skinny) {
  if (!skinny) return gemm_splits(h);
  // about 256 workgroups: a column tile per thread block carries enough work
  // that more splits only add partial traffic
  const uint64_t tiles = gemm_tiles(h, true);
  const uint64_t kchunks = (h.K + SK_KC - 1) / SK_KC;
  uint64_t s = std::max<uint64_t>(1, 256 / std::max<uint64_t>(tiles, 1));
  s = std::min<uint64_t>(s, kchunks);
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(s, 65535));
}

uint64_t gemm_k_per_split(const GemmArgs &h, uint32_t splits, bool skinny) {
  const uint64_t kc = skinny ? SK_KC : KC;
  const uint64_t kchunks = (h.K + kc - 1) / kc;
  return ((kchunks + splits - 1) / splits) * kc;
}

// The MFMA tile kernel of precision mode `mode` (0 fp64, 1 fp32, 2 fp32
// hi/lo) with `lds` bytes of factor tables; batch: the job list, else one
// contraction.
hipError_t gemm_launch(int mode, bool gen, dim3 g, size_t lds, hipStream_t s, const GemmJob *jobs, uint32_t n_jobs,
                       const GemmArgs *args, uint64_t k_per_split, double *partial, double *out) {
  if (lds > 96 * 1024) return hipErrorInvalidValue;
#define CCUT_GEMM(M_, G_)                                                                                     \
  do {                                                                                                        \
    const void *fn = jobs ? (const void *)gemm_batch_kernel<M_, G_> : (const void *)gemm_kernel<M_, G_>;     \
    if (lds) {                                                                                                \
      hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);           \
      if (e != hipSuccess) return e;                                                                          \
    }                                                                                                         \
    if (jobs)                                                                                                 \
      hipLaunchKernelGGL((gemm_batch_kernel<M_, G_>), g, dim3(GEMM_THREADS), lds, s, jobs, n_jobs);          \
    else                                                                                                      \
      hipLaunchKernelGGL((gemm_kernel<M_, G_>), g, dim3(GEMM_THREADS), lds, s, args, k_per_split, partial, out); \
  } while (0)
  switch (mode * 2 + (gen ? 1 : 0)) {
    case 0: CCUT_GEMM(0, false); break;
    case 1: CCUT_GEMM(0, true); break;
    case 2: CCUT_GEMM(1, false); break;
    case 3: CCUT_GEMM(1, true); break;
    case 4: CCUT_GEMM(2, false); break;
    default: CCUT_GEMM(2, true); break;
  }
#undef CCUT_GEMM
  return hipGetLastError();
}

size_t gemm_fac_lds(const GemmArgs &h) { return (size_t)(fac_words(h, h.L) + fac_words(h, h.R)) * sizeof(double); }

// Whether contraction h needs the general tile kernel (a side that is not
// one fragment read directly).
bool gemm_general(const GemmArgs &h) {
  auto direct = [&](const GemmSide &S) { return S.n == 1 && !h.terms && S.shift[0] == 0 && h.ident[S.frag[0]]; };
  return !direct(h.L) || !direct(h.R);
}

hipError_t launch_gemm_batch(const GemmJob *d_jobs, uint32_t n_jobs, uint64_t total_wg, uint64_t total_rwg, int mode,
                             bool gen, size_t lds, uint32_t skinny_rows, uint32_t skinny_cpt, hipStream_t s) {
  if (n_jobs == 0 || total_wg == 0) return hipSuccess;
  if (total_wg > 0x7FFFFFFFull || total_rwg > 0x7FFFFFFFull) return hipErrorInvalidValue;
  hipError_t e;
  if (skinny_rows)
    e = skinny_dispatch(skinny_rows, skinny_cpt, dim3((unsigned)total_wg), s, d_jobs, n_jobs, nullptr, 0, nullptr,
                        nullptr);
  else
    e = gemm_launch(mode, gen, dim3((unsigned)total_wg), gen ? lds : 0, s, d_jobs, n_jobs, nullptr, 0, nullptr,
                    nullptr);
  if (e != hipSuccess || total_rwg == 0) return e;  // (one-split jobs wrote their outputs)
  hipLaunchKernelGGL(gemm_reduce_batch_kernel, dim3((unsigned)total_rwg), dim3(256), 0, s, d_jobs, n_jobs);
  return hipGetLastError();
}

hipError_t launch_recombine_gemm(const GemmArgs &h, const GemmArgs *d_args, bool fp32, double *partial,
                                 uint32_t splits, double *out, hipStream_t s, bool skinny) {
  const uint32_t tiles = gemm_tiles(h, skinny);
  const uint64_t k_per_split = gemm_k_per_split(h, splits, skinny);
  if (skinny) {
    const hipError_t e = skinny_dispatch(h.M, skinny_cols(h), dim3(tiles, splits), s, nullptr, 0, d_args,
                                         k_per_split, partial, splits == 1 ? out : nullptr);
    if (e != hipSuccess || splits == 1) return e;
  } else {
    const bool gen = gemm_general(h);
    const hipError_t e = gemm_launch(fp32 ? (h.lo_parts ? 2 : 1) : 0, gen, dim3(tiles, splits),
                                     gen ? gemm_fac_lds(h) : 0, s, nullptr, 0, d_args, k_per_split, partial,
                                     splits == 1 ? out : nullptr);
    if (e != hipSuccess || splits == 1) return e;
  }
  const uint64_t MN = (uint64_t)h.M * h.N;
  hipLaunchKernelGGL(gemm_reduce_kernel, dim3((unsigned)((MN + 255) / 256)), dim3(256), 0, s, d_args, partial,
                     splits, out);
  return hipGetLastError();
}

}  // namespace ccut

// Exact Pauli-basis tensors of Clifford fragments in the Heisenberg picture
// (the Clifford-specific cutting optimisation the paper outlines in Sec. IX:
// Clifford expectations are -1, 0 or +1 and most Pauli terms vanish).
//
// For a Clifford fragment U with quantum inputs (prepared as the operator
// P_in), circuit inputs |0> and a measured set, the Pauli-basis entry is
//   tau[S; P_out, P_in] = Tr[(Z_S (x) Q_out) U rho_in U^dag]
//                       = Tr[O rho_in],   O = U^dag (Z_S (x) Q_out) U,
// and with O = (-1)^s sigma_1 (x) ... (x) sigma_m:
//   Tr[O rho_in] = (-1)^s 2^#in [sigma|inputs == P_in] [sigma|circuit inputs in {I, Z}].
// The marginal tensor is T[b; P] = 2^-r sum_S (-1)^{b.S} tau[S; P] (the
// projector onto outcome b is 2^-r sum_S (-1)^{b.S} Z_S), a Walsh-Hadamard
// transform over subsets S of the r requested outputs.  No variant is
// enumerated: only the r requested Z's and the X, Z of each quantum output
// are carried back through the fragment once.
#include <algorithm>

#include "common.hpp"

namespace ccut {

namespace {

// Shared pass of many fragments' rows: the descriptor array in the global
// address space, read through a reference.
typedef __attribute__((address_space(1))) const FragDev g_FragDevH;

// The row pass bit-sliced: column q of the x (z) parts holds bit q of
// 64 rows per word, so a gate reads and writes only its qubits' column
// words and applies its rule to 64 rows with a few 64-bit operations.  The
// stream comes in layers of ops on disjoint qubits.  Lane l works on row
// word w = l mod RWp (RWp = RW rounded up to a power of two) and, within a
// layer, on op l / RWp of each group of 64 / RWp ops, so a layer costs one
// round trip through LDS instead of one per gate.  Each lane XORs the sign
// changes of its ops into one private word (XOR commutes, and an op reads
// the columns as they are before it: earlier layers are complete and its
// own layer never touches its qubits); one reduction over the lanes of each
// row word adds them up at the end.  One wave, so LDS accesses complete in
// issue order; a compiler fence keeps the layers in order.  Columns live in
// LDS ([m][RW] for x, then for z); rows are transposed in (or start as the
// identity tableau when `in` is null) and back out in the (x[W], z[W],
// sign) row layout.  At most 1024 rows per wave.
constexpr uint32_t kSlicedRows = 1024;
constexpr uint32_t kOpStage = 1024;  // op words staged in LDS (a layer has at most 512)
constexpr uint32_t kLayStage = 256;  // layer offsets staged in LDS

// Fill dst[0, CAP) from src[0, n) (zeros past n) with all loads of a lane
// issued before its first store, so the copy costs one memory latency
// rather than one per word (one wave).
template <uint32_t CAP>
__device__ inline void stage_words(uint32_t *dst, const uint32_t *src, uint32_t n, uint32_t lane) {
  constexpr uint32_t K = (CAP + 63) / 64;
  uint32_t t[K];
#pragma unroll
  for (uint32_t k = 0; k < K; ++k) {
    const uint32_t i = lane + 64 * k;
    t[k] = i < n && i < CAP ? src[i] : 0u;
  }
#pragma unroll
  for (uint32_t k = 0; k < K; ++k)
    if (lane + 64 * k < CAP) dst[lane + 64 * k] = t[k];
}

// NW waves per workgroup: a layer's ops are spread over all 64 NW lanes and
// the waves meet at a barrier after each layer (a lane reads columns other
// waves wrote in the previous layer); wave 0 stages op words and layer
// offsets and transposes rows in and out, and the lanes' sign shares are
// XOR-reduced within each wave, then across the waves through LDS.  NW = 1:
// no barriers (one wave's LDS accesses complete in issue order).
template <uint32_t NW, class D>
__device__ void rows_sliced_body(const D &F, uint32_t W, const uint64_t *__restrict__ in, uint64_t *__restrict__ out,
                                 uint32_t n_rows, uint64_t *cols) {
  constexpr uint32_t T = 64 * NW;
  const uint32_t m = F.m;
  const uint32_t RW = (n_rows + 63) / 64;
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
  uint32_t lg = 0;
  while ((1u << lg) < RW) ++lg;
  const uint32_t RWp = 1u << lg, w = tid & (RWp - 1), o = tid >> lg, per = T >> lg;
  uint64_t *Xc = cols, *Zc = cols + (size_t)m * RW;
  uint32_t *sops = reinterpret_cast<uint32_t *>(Zc + (size_t)m * RW);
  const uint32_t RS = 2 * W + 1;  // row stride in words
  uint64_t sg = 0;  // this lane's share of sign word w
  auto sync = [] {
    if (NW > 1) __syncthreads();
  };
  if (!in) {
    for (uint32_t idx = tid; idx < m * RW; idx += T) {  // X_r for rows r < m, then Z_{r - m}
      const uint32_t q = idx / RW, iw = idx % RW;
      Xc[idx] = q >> 6 == iw ? 1ull << (q & 63) : 0ull;
      Zc[idx] = (m + q) >> 6 == iw ? 1ull << ((m + q) & 63) : 0ull;
    }
  } else if (wave == 0) {
    // transpose in, 64 rows at a time: lane l loads row 64 iw + l whole,
    // and column word (q, iw) is the ballot of bit q over the lanes
    for (uint32_t iw = 0; iw < RW; ++iw) {
      const uint32_t r = 64 * iw + lane;
      const bool ok = r < n_rows;
      const uint64_t *row = in + (size_t)(ok ? r : 0) * RS;
      uint64_t xr[8], zr[8];
#pragma unroll
      for (uint32_t k = 0; k < 8; ++k) {
        xr[k] = ok && k < W ? row[k] : 0ull;
        zr[k] = ok && k < W ? row[W + k] : 0ull;
      }
      const uint64_t sw = __ballot(ok && (row[2 * W] & 1ull));
      if (lane == iw) sg = sw;  // lane iw starts with sign word iw
#pragma unroll
      for (uint32_t k = 0; k < 8; ++k) {
        if (k >= W) break;
        const uint32_t nq = 64 * k < m ? min(64u, m - 64 * k) : 0u;
        for (uint32_t i = 0; i < nq; ++i) {
          const uint64_t cx = __ballot((xr[k] >> i) & 1ull), cz = __ballot((zr[k] >> i) & 1ull);
          if (lane == i) {
            Xc[(size_t)(64 * k + i) * RW + iw] = cx;
            Zc[(size_t)(64 * k + i) * RW + iw] = cz;
          }
        }
      }
    }
  }
  const bool live = w < RW;
  __syncthreads();
  // Layer offsets are staged in LDS too (without offsets every op is a
  // layer of its own).  One layer of lookahead: the next layer's end offset
  // and this lane's first op word of the next layer are read before the
  // current layer's column traffic, so only the column reads wait on LDS.
  // Op words are restaged when the next layer (at most 512 ops) might not
  // lie inside the staged window.
  uint32_t *slay = sops + kOpStage;
  const uint32_t *lay = F.layers;
  const uint32_t n_layers = lay ? F.n_layers : F.n_ops;
  uint32_t stage0 = 0;
  if (wave == 0) stage_words<kOpStage>(sops, F.ops, F.n_ops, lane);
  uint32_t s0 = 0;
  for (uint32_t L0 = 0; L0 < n_layers; L0 += kLayStage) {
    const uint32_t nl = min(kLayStage, n_layers - L0);
    if (wave == 0) {
      if (lay) {
        stage_words<kLayStage + 1>(slay, lay + L0, nl + 1, lane);
      } else {
        for (uint32_t i = lane; i <= nl; i += 64) slay[i] = L0 + i;
      }
    }
    sync();  // the staged words (and, the first time, the op window) are in place
    uint32_t v_s1 = slay[1];
    uint32_t v_wd = sops[s0 + o - stage0];  // this lane's first op word of the current layer
    for (uint32_t L = 0; L < nl; ++L) {
      const uint32_t s1 = __builtin_amdgcn_readfirstlane(v_s1);
      const uint32_t wd0 = v_wd;
      const bool keep = s1 + 512 <= stage0 + kOpStage;  // the next layer is inside the window
      uint32_t v_s1n = 0, v_wdn = 0;
      if (L + 2 <= nl) v_s1n = slay[L + 2];
      if (keep) v_wdn = sops[s1 + o - stage0];
      for (uint32_t c0 = s0 + o; c0 < s1; c0 += per) {
        if (!live) continue;
        const uint32_t wd = c0 == s0 + o ? wd0 : sops[c0 - stage0];
        const uint32_t kind = op_kind(wd), a = op_q0(wd), b = op_q1(wd);
        uint64_t *xa = Xc + (size_t)a * RW + w, *za = Zc + (size_t)a * RW + w;
        if (kind == G_CX || kind == G_CZ) {
          uint64_t *xb = Xc + (size_t)b * RW + w, *zb = Zc + (size_t)b * RW + w;
          const uint64_t x1 = *xa, z1 = *za, x2 = *xb, z2 = *zb;
          if (kind == G_CX) {
            sg ^= x1 & z2 & ~(x2 ^ z1);
            *xb = x2 ^ x1;
            *za = z1 ^ z2;
          } else {
            sg ^= x1 & x2 & (z1 ^ z2);
            *za = z1 ^ x2;
            *zb = z2 ^ x1;
          }
        } else {
          const C1Map g = c1_decode(b);
          const uint64_t x = *xa, z = *za;
          sg ^= (x & (0ull - g.al)) ^ (z & (0ull - g.be)) ^ (x & z & (0ull - g.ga));
          *xa = (x & (0ull - g.m00)) ^ (z & (0ull - g.m01));
          *za = (x & (0ull - g.m10)) ^ (z & (0ull - g.m11));
        }
      }
      asm volatile("" ::: "memory");
      sync();  // every wave is done with this layer's columns (and op words)
      if (!keep) {  // restage from the next layer's start (in issue order after this layer's reads)
        stage0 = s1;
        if (wave == 0) stage_words<kOpStage>(sops, F.ops + s1, F.n_ops - s1, lane);
        sync();
        v_wdn = sops[o];
      }
      s0 = s1;
      v_s1 = v_s1n;
      v_wd = v_wdn;
    }
    sync();  // every wave has read this stage's layer offsets
  }
  // sign word w: XOR of the shares of every lane on row word w (lane w of
  // wave 0 ends with it)
  for (uint32_t off = RWp; off < 64; off <<= 1) sg ^= __shfl_xor(sg, off);
  __syncthreads();
  if (NW > 1) {
    uint64_t *red = reinterpret_cast<uint64_t *>(sops);  // the op window is no longer read
    if (lane < RWp) red[wave * 64 + lane] = sg;
    __syncthreads();
    if (wave == 0 && lane < RWp)
      for (uint32_t v = 1; v < NW; ++v) sg ^= red[v * 64 + lane];
  }
  if (wave != 0) return;
  // transpose out, 64 rows at a time: lane l gathers row 64 rw + l from the
  // column words (each read is the same address for every lane)
  for (uint32_t rw = 0; rw < RW; ++rw) {
    const uint32_t r = 64 * rw + lane;
    for (uint32_t wq = 0; wq < W; ++wq) {
      const uint32_t nq = 64 * wq < m ? min(64u, m - 64 * wq) : 0u;
      uint64_t xw = 0, zw = 0;
#pragma unroll 8
      for (uint32_t i = 0; i < nq; ++i) {
        const size_t c = (size_t)(64 * wq + i) * RW + rw;
        xw |= ((Xc[c] >> lane) & 1ull) << i;
        zw |= ((Zc[c] >> lane) & 1ull) << i;
      }
      if (r < n_rows) {
        out[(size_t)r * RS + wq] = xw;
        out[(size_t)r * RS + W + wq] = zw;
      }
    }
  }
  for (uint32_t rw = 0; rw < RW; ++rw) {
    const uint64_t word = __shfl(sg, rw);
    const uint32_t r = 64 * rw + lane;
    if (r < n_rows) out[(size_t)r * RS + 2 * W] = (word >> lane) & 1ull;
  }
}

// Block x carries rows [1024 x, 1024 x + 1024) (rows are independent).
__global__ __launch_bounds__(64) void rows_sliced_kernel(const FragDev F, uint32_t W, const uint64_t *__restrict__ in,
                                                          uint64_t *__restrict__ out, uint32_t n_rows) {
  extern __shared__ uint64_t cols[];
  const uint32_t r0 = blockIdx.x * kSlicedRows;
  const size_t RS = 2 * W + 1;
  rows_sliced_body<1>(F, W, in ? in + r0 * RS : nullptr, out + r0 * RS, min(kSlicedRows, n_rows - r0), cols);
}

// Carry-back of many fragments' rows: block x carries job x's n_rows input
// rows (row width W words per half) through its descriptor's stream, with
// kCarryWaves waves spreading each layer's ops.
constexpr uint32_t kCarryWaves = 4;
__global__ __launch_bounds__(64 * kCarryWaves) void carry_batch_kernel(const FragDev *__restrict__ descs,
                                                          const CarryJob *__restrict__ jobs,
                                                          const uint64_t *__restrict__ in, uint64_t *__restrict__ out) {
  extern __shared__ uint64_t cols[];
  const CarryJob &J = jobs[blockIdx.x];
  const g_FragDevH &F = ((const g_FragDevH *)descs)[J.desc];
  rows_sliced_body<kCarryWaves>(F, J.W, in + J.in_off, out + J.out_off, J.n_rows, cols);
}

struct HeisArgs {
  uint32_t m, W, n_axes, n_in, n_out, r;
  uint32_t axis_side[kMaxAxes];
  uint32_t axis_local[kMaxAxes];
  uint64_t cin_mask[8];  // local qubits that are circuit inputs
  uint32_t n_str;        // Z-string mode: number of string rows (0 = marginal mode)
};

// Phase-tracked product: P = i^a X^x Z^z.
template <int W>
struct PAcc {
  uint64_t x[W], z[W];
  uint32_t a;
};

template <int W>
__device__ inline void pmul(PAcc<W> &L, const uint64_t *R) {  // L <- L * R (R a Hermitian row)
  uint32_t cross = 0, pr = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    cross += __popcll(L.z[w] & R[w]);
    pr += __popcll(R[w] & R[W + w]);
  }
  L.a = (L.a + 2u * (uint32_t)R[2 * W] + pr + 2u * cross) & 3u;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    L.x[w] ^= R[w];
    L.z[w] ^= R[W + w];
  }
}

template <int W>
__device__ inline uint32_t pbit(const uint64_t (&v)[W], uint32_t q) {
  uint64_t word = v[0];
#pragma unroll
  for (int w = 1; w < W; ++w)
    if ((q >> 6) == (uint32_t)w) word = v[w];
  return (uint32_t)(word >> (q & 63)) & 1u;
}

// One thread per (S or string, P_out combination).  rows: for the marginal
// mode the r requested Z images followed by (X_c, Z_c) images per output;
// for the string mode n_str string images followed by the output images.
// tau[p_f][col] (zero-filled by the caller) receives the single nonzero
// entry of this (col, P_out) if the circuit-input condition holds.
template <int W>
__global__ void tau_kernel(const HeisArgs A, const uint64_t *__restrict__ rows, double *__restrict__ tau,
                           uint64_t ncols) {
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t n_pout = 1ull << (2 * A.n_out);
  if (t >= ncols * n_pout) return;
  const uint64_t col = t % ncols;
  const uint64_t pc = t / ncols;
  const uint32_t RW = 2 * W + 1;
  PAcc<W> acc;
#pragma unroll
  for (int w = 0; w < W; ++w) acc.x[w] = acc.z[w] = 0;
  acc.a = 0;
  uint32_t out_base;
  if (A.n_str == 0) {
    for (uint32_t j = 0; j < A.r; ++j)
      if ((col >> j) & 1ull) pmul<W>(acc, rows + (size_t)j * RW);
    out_base = A.r;
  } else {
    pmul<W>(acc, rows + (size_t)col * RW);
    out_base = A.n_str;
  }
  // output Paulis, in output-axis order; Y = i X Z
  uint32_t oc = 0;
  uint64_t pf = 0;
  for (uint32_t j = 0; j < A.n_axes; ++j) {
    if (A.axis_side[j] != 0) continue;
    const uint32_t P = (uint32_t)((pc >> (2 * oc)) & 3ull);  // I, X, Y, Z
    const uint64_t *rx = rows + (size_t)(out_base + 2 * oc) * RW;
    const uint64_t *rz = rx + RW;
    if (P == 1) pmul<W>(acc, rx);
    if (P == 3) pmul<W>(acc, rz);
    if (P == 2) {
      acc.a = (acc.a + 1u) & 3u;
      pmul<W>(acc, rx);
      pmul<W>(acc, rz);
    }
    pf |= (uint64_t)P << (2 * j);
    ++oc;
  }
  // circuit inputs must carry I or Z
#pragma unroll
  for (int w = 0; w < W; ++w)
    if (acc.x[w] & A.cin_mask[w]) return;
  for (uint32_t j = 0; j < A.n_axes; ++j) {
    if (A.axis_side[j] != 1) continue;
    const uint32_t q = A.axis_local[j];
    const uint32_t xq = pbit<W>(acc.x, q), zq = pbit<W>(acc.z, q);
    const uint32_t P = xq ? (zq ? 2u : 1u) : (zq ? 3u : 0u);
    pf |= (uint64_t)P << (2 * j);
  }
  uint32_t pxz = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) pxz += __popcll(acc.x[w] & acc.z[w]);
  const uint32_t sgn = ((acc.a - pxz) & 3u) >> 1;  // acc is Hermitian: a - x.z in {0, 2}
  tau[pf * ncols + col] = ldexp(sgn ? -1.0 : 1.0, (int)A.n_in);
}

// T[row][b] = 2^-r sum_S (-1)^{b.S} tau[row][S]: in-place WHT per row in LDS.
constexpr int kWht = 256;
__global__ __launch_bounds__(kWht) void subset_wht_kernel(double *__restrict__ data, uint32_t r) {
  extern __shared__ double w[];
  const uint32_t n = 1u << r;
  double *row = data + (uint64_t)blockIdx.x * n;
  for (uint32_t i = threadIdx.x; i < n; i += kWht) w[i] = row[i];
  __syncthreads();
  for (uint32_t s = 0; s < r; ++s) {
    for (uint32_t k = threadIdx.x; k < n / 2; k += kWht) {
      const uint32_t i0 = ((k >> s) << (s + 1)) | (k & ((1u << s) - 1)), i1 = i0 | (1u << s);
      const double a = w[i0], b = w[i1];
      w[i0] = a + b;
      w[i1] = a - b;
    }
    __syncthreads();
  }
  for (uint32_t i = threadIdx.x; i < n; i += kWht) row[i] = ldexp(w[i], -(int)r);
}

// The same for rows of at most 64 entries: one wave per row, entry l in
// lane l, the butterflies through lane exchanges (the same additions and
// subtractions in the same order as the LDS version), four rows per
// workgroup, coalesced row reads and writes.
__global__ __launch_bounds__(256) void subset_wht_wave_kernel(double *__restrict__ data, uint32_t r, uint64_t nrows) {
  const uint64_t row = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= nrows) return;  // whole waves leave together
  const uint32_t l = threadIdx.x & 63, n = 1u << r;
  double v = l < n ? data[row * n + l] : 0.0;
  for (uint32_t s = 0; s < r; ++s) {
    const double p = __shfl_xor(v, 1 << s);
    v = ((l >> s) & 1u) ? p - v : v + p;  // the pair (a, b) becomes (a + b, a - b)
  }
  if (l < n) data[row * n + l] = ldexp(v, -(int)r);
}

__global__ void fill_zero_kernel(double *p, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

template <int W>
hipError_t run_w(const FragDev &F, const HeisArgs &A, const uint64_t *rows_in, uint64_t *rows_out, uint32_t n_rows,
                 double *tau, uint64_t ncols, hipStream_t s) {
  hipError_t e;
  if (n_rows && (e = launch_rows(F, W, rows_in, rows_out, n_rows, s)) != hipSuccess) return e;
  const uint64_t total_tau = ncols << (2 * A.n_axes);
  hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)std::min<uint64_t>((total_tau + 255) / 256, 65536)), dim3(256),
                     0, s, tau, total_tau);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const uint64_t nt = ncols << (2 * A.n_out);
  hipLaunchKernelGGL((tau_kernel<W>), dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, A, rows_out, tau, ncols);
  return hipGetLastError();
}

}  // namespace

// rows_in: host-built Pauli rows [n_rows][2W+1] with W = words(m) rounded up
// to {1, 2, 4, 8}; see k_heis layout.  Marginal mode (n_str == 0): rows are
// r requested Z's then (X_c, Z_c) per output axis; tau is [4^n_axes][2^r] and
// is turned into T[p_f][b] in place.  String mode: rows are n_str strings then
// the output pairs; tau is [4^n_axes][n_str] = t_f[p_f][string].
size_t rows_sliced_lds(uint32_t m, uint32_t n_rows) {
  return (size_t)2 * m * ((n_rows + 63) / 64) * 8 + (kOpStage + kLayStage + 1) * 4;
}

hipError_t launch_rows(const FragDev &F, uint32_t W, const uint64_t *in, uint64_t *out, uint32_t n_rows,
                       hipStream_t s) {
  if (n_rows == 0) return hipSuccess;
  if ((W != 1 && W != 2 && W != 4 && W != 8) || F.m > 64 * W || (!in && n_rows > kSlicedRows))
    return hipErrorInvalidValue;
  const size_t lds = rows_sliced_lds(F.m, std::min(n_rows, kSlicedRows));
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute((const void *)rows_sliced_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(rows_sliced_kernel, dim3((n_rows + kSlicedRows - 1) / kSlicedRows), dim3(64), lds, s, F, W, in,
                     out, n_rows);
  return hipGetLastError();
}

hipError_t launch_carry_batch(const FragDev *descs, const CarryJob *jobs, uint32_t n_jobs, uint32_t max_m,
                              uint32_t max_rows, const uint64_t *in, uint64_t *out, hipStream_t s) {
  if (n_jobs == 0) return hipSuccess;
  if (max_rows > kSlicedRows) return hipErrorInvalidValue;
  const size_t lds = rows_sliced_lds(max_m, max_rows);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute((const void *)carry_batch_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(carry_batch_kernel, dim3(n_jobs), dim3(64 * kCarryWaves), lds, s, descs, jobs, in, out);
  return hipGetLastError();
}

hipError_t launch_heisenberg(const FragDev &F, uint32_t W, uint32_t n_in, uint32_t n_out, uint32_t r,
                             uint32_t n_str, const uint64_t *cin_mask, const uint64_t *rows_in, uint64_t *rows_out,
                             uint32_t n_rows, double *tau, hipStream_t s) {
  HeisArgs A{};
  A.m = F.m;
  A.W = W;
  A.n_axes = F.n_axes;
  A.n_in = n_in;
  A.n_out = n_out;
  A.r = r;
  A.n_str = n_str;
  for (uint32_t j = 0; j < F.n_axes; ++j) {
    A.axis_side[j] = F.axis_side[j];
    A.axis_local[j] = F.axis_local[j];
  }
  for (uint32_t w = 0; w < 8; ++w) A.cin_mask[w] = w < W ? cin_mask[w] : 0;
  const uint64_t ncols = n_str ? n_str : (1ull << r);
  hipError_t e;
  switch (W) {
    case 1: e = run_w<1>(F, A, rows_in, rows_out, n_rows, tau, ncols, s); break;
    case 2: e = run_w<2>(F, A, rows_in, rows_out, n_rows, tau, ncols, s); break;
    case 4: e = run_w<4>(F, A, rows_in, rows_out, n_rows, tau, ncols, s); break;
    case 8: e = run_w<8>(F, A, rows_in, rows_out, n_rows, tau, ncols, s); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess || n_str) return e;
  const uint64_t nrows = 1ull << (2 * F.n_axes);
  if (r == 0) return hipSuccess;
  if (r <= 6) {
    for (uint64_t r0 = 0; r0 < nrows; r0 += (1ull << 32)) {
      const uint64_t cnt = std::min<uint64_t>(nrows - r0, 1ull << 32);
      hipLaunchKernelGGL(subset_wht_wave_kernel, dim3((unsigned)((cnt + 3) / 4)), dim3(256), 0, s, tau + (r0 << r), r,
                         cnt);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
  }
  for (uint64_t r0 = 0; r0 < nrows; r0 += (1ull << 30)) {
    const uint64_t cnt = std::min<uint64_t>(nrows - r0, 1ull << 30);
    hipLaunchKernelGGL(subset_wht_kernel, dim3((unsigned)cnt), dim3(kWht), (size_t(1) << r) * 8, s,
                       tau + (r0 << r), r);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace ccut

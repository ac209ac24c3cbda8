// Learned importance proposal over the 4^k cut terms of the recombination
// sum (Sec. V-C; its cost grows as 4^k, Sec. III-B): a small ReLU MLP maps
// per-term features to a predicted log-weight, trained and evaluated here
// with BF16 MFMA products and fp32 accumulation; the proposal
// q = (1 - eps) softmax + eps / K, its integer CDF, Philox inverse-CDF term
// sampling, and the per-term inputs (features, labels, support) computed
// from the fragment tensors.
//
// MFMA lane layout of v_mfma_f32_16x16x16_bf16 (checked on gfx950): lane l
// supplies A[row l % 16][k 4 (l / 16) + i] and B[k 4 (l / 16) + i][col l % 16]
// for i < 4; accumulator register g holds D[row 4 (l / 16) + g][col l % 16].
#include <cmath>
#include <mutex>

#include "ccut.h"
#include "common.hpp"

namespace ccut {

namespace {

typedef short short4v __attribute__((ext_vector_type(4)));
typedef float float4v __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// fp32 -> bf16, round to nearest even (NaN kept quiet)
__device__ inline uint16_t f2bf(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x7FFFFFu)) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

constexpr int MG_T = 64, MG_K = 32, MG_PAD = 8, MG_THREADS = 256;

// C[M x N] = sum_k A(m, k) B(k, n), A(m, k) = A[m sam + k sak],
// B(k, n) = B[k sbk + n sbn] (bf16), fp32 accumulation; one of the
// strides of each operand is 1.  Rows m >= M read as zero and are not
// written; N % 64 == 0 and K % 32 == 0.
template <int EPI>
__global__ __launch_bounds__(MG_THREADS) void mlp_gemm_kernel(const MlpGemm g) {
  __shared__ __attribute__((aligned(16))) uint16_t As[MG_T][MG_K + MG_PAD];  // [m][k]
  __shared__ __attribute__((aligned(16))) uint16_t Bs[MG_T][MG_K + MG_PAD];  // [n][k]
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint64_t m0 = (uint64_t)blockIdx.x * MG_T;
  const uint32_t n0 = blockIdx.y * MG_T;
  const uint32_t wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  float4v acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = float4v{0.f, 0.f, 0.f, 0.f};
  for (uint32_t k0 = 0; k0 < g.K; k0 += MG_K) {
    // A tile: 64 rows x 32 k, eight contiguous elements per thread
    if (g.sak == 1) {
      const uint32_t mm = tid >> 2, kc = (tid & 3) * 8;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (m0 + mm < g.M) v = *(const uint4 *)(g.A + (m0 + mm) * g.sam + k0 + kc);
      *(uint4 *)&As[mm][kc] = v;
    } else {
      const uint32_t kk = tid >> 3, mc = (tid & 7) * 8;
      uint16_t e[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      if (m0 + mc + 8 <= g.M) {
        const uint4 v = *(const uint4 *)(g.A + (m0 + mc) + (uint64_t)(k0 + kk) * g.sak);
        const uint16_t *pv = (const uint16_t *)&v;
#pragma unroll
        for (int t = 0; t < 8; ++t) e[t] = pv[t];
      } else {
        for (int t = 0; t < 8; ++t)
          if (m0 + mc + t < g.M) e[t] = g.A[(m0 + mc + t) + (uint64_t)(k0 + kk) * g.sak];
      }
#pragma unroll
      for (int t = 0; t < 8; ++t) As[mc + t][kk] = e[t];
    }
    // B tile: 32 k x 64 columns, stored [n][k]
    if (g.sbk == 1) {
      const uint32_t nn = tid >> 2, kc = (tid & 3) * 8;
      *(uint4 *)&Bs[nn][kc] = *(const uint4 *)(g.B + (uint64_t)(n0 + nn) * g.sbn + k0 + kc);
    } else {
      const uint32_t kk = tid >> 3, nc = (tid & 7) * 8;
      const uint4 v = *(const uint4 *)(g.B + (uint64_t)(k0 + kk) * g.sbk + n0 + nc);
      const uint16_t *pv = (const uint16_t *)&v;
#pragma unroll
      for (int t = 0; t < 8; ++t) Bs[nc + t][kk] = pv[t];
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < MG_K; ks += 16) {
      short4v a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = *(const short4v *)&As[wm + 16 * i + (lane & 15)][ks + 4 * (lane >> 4)];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = *(const short4v *)&Bs[wn + 16 * j + (lane & 15)][ks + 4 * (lane >> 4)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint64_t m = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
        const uint32_t n = n0 + wn + 16 * j + (lane & 15);
        if (m >= g.M) continue;
        float v = acc[i][j][r];
        if (EPI == MLP_EPI_F32) {
          ((float *)g.C)[m * g.ldc + n] = v;
        } else if (EPI == MLP_EPI_BIAS_RELU) {
          v = fmaxf(v + g.bias[n], 0.f);
          ((uint16_t *)g.C)[m * g.ldc + n] = f2bf(v);
        } else {  // MLP_EPI_MASK: gradient through the ReLU of the layer output stored in mask
          v = bf2f(g.mask[m * g.ldm + n]) > 0.f ? v : 0.f;
          ((uint16_t *)g.C)[m * g.ldc + n] = f2bf(v);
        }
      }
}

// y[m] = scale (b + sum_n H[m][n] w[n]); 32 lanes per row, eight elements per lane,
// summed in a fixed butterfly order.
__global__ void head_forward_kernel(const uint16_t *__restrict__ H, uint32_t width, uint64_t rows,
                                    const uint16_t *__restrict__ w, const float *__restrict__ b, float scale,
                                    float *__restrict__ y) {
  const uint64_t row = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 5;
  const uint32_t l = threadIdx.x & 31;
  float s = 0.f;
  if (row < rows)
    for (uint32_t c = l * 8; c < width; c += 256) {
      const uint4 hv = *(const uint4 *)(H + row * width + c);
      const uint4 wv = *(const uint4 *)(w + c);
      const uint16_t *hp = (const uint16_t *)&hv, *wp = (const uint16_t *)&wv;
#pragma unroll
      for (int t = 0; t < 8; ++t) s += bf2f(hp[t]) * bf2f(wp[t]);
    }
#pragma unroll
  for (int o = 16; o > 0; o >>= 1) s += __shfl_xor(s, o, 32);
  if (row < rows && l == 0) y[row] = scale * (s + b[0]);
}

// Loss terms and the output-layer backward: r = y - t, dy = 2 r / B,
// sq[m] = r^2, dZ[m][n] = dy w[n] [H[m][n] > 0] (bf16).
__global__ void head_backward_kernel(const uint16_t *__restrict__ H, uint32_t width, uint64_t rows,
                                     const uint16_t *__restrict__ w, const float *__restrict__ y,
                                     const float *__restrict__ t, float inv_b2, float *__restrict__ dy,
                                     float *__restrict__ sq, uint16_t *__restrict__ dZ) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * width) return;
  const uint64_t m = i / width;
  const uint32_t n = (uint32_t)(i % width);
  const float r = y[m] - t[m];
  const float d = r * inv_b2;
  if (n == 0) {
    dy[m] = d;
    sq[m] = r * r;
  }
  dZ[i] = f2bf(bf2f(H[i]) > 0.f ? d * bf2f(w[n]) : 0.f);
}

// Column sums out[n] = sum_m s[m] X[m][n] (s == nullptr: 1) in two
// ordered passes: per-chunk partials, then the chunks in order.
constexpr uint32_t kColChunk = 256;
__global__ void colsum_partial_kernel(const uint16_t *__restrict__ X, uint32_t width, uint64_t rows,
                                      const float *__restrict__ s, float *__restrict__ part) {
  const uint32_t n = threadIdx.x;
  if (n >= width) return;
  const uint64_t r0 = (uint64_t)blockIdx.x * kColChunk;
  const uint64_t r1 = r0 + kColChunk < rows ? r0 + kColChunk : rows;
  float acc = 0.f;
  for (uint64_t m = r0; m < r1; ++m) acc += (s ? s[m] : 1.f) * bf2f(X[m * width + n]);
  part[(uint64_t)blockIdx.x * width + n] = acc;
}
__global__ void colsum_final_kernel(const float *__restrict__ part, uint32_t width, uint32_t chunks,
                                    float *__restrict__ out) {
  const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= width) return;
  float acc = 0.f;
  for (uint32_t c = 0; c < chunks; ++c) acc += part[(uint64_t)c * width + n];
  out[n] = acc;
}

// *out = sum of x[0..n) (one workgroup, fixed-order tree)
__global__ __launch_bounds__(256) void vsum_kernel(const float *__restrict__ x, uint64_t n, float *__restrict__ out) {
  __shared__ float red[256];
  float acc = 0.f;
  for (uint64_t i = threadIdx.x; i < n; i += 256) acc += x[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (uint32_t w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// Adam (Kingma & Ba) on the flat fp32 parameters; c1 = 1 - b1^t,
// c2 = 1 - b2^t.  Also refreshes the bf16 copy used by the products.
__global__ void adam_kernel(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ v, uint16_t *__restrict__ pb, uint64_t n, float lr, float b1,
                            float b2, float c1, float c2, float eps) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float np = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  p[i] = np;
  pb[i] = f2bf(np);
}

__global__ void to_bf16_kernel(const float *__restrict__ p, uint16_t *__restrict__ pb, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) pb[i] = f2bf(p[i]);
}

// Mini-batch rows: row i of step `step` is row (philox bits mod n) of the
// data set, or row i itself when the batch covers the data set in order.
__global__ void gather_rows_kernel(const uint16_t *__restrict__ X, const float *__restrict__ y, uint64_t n,
                                   uint32_t width, uint32_t batch, uint32_t step, uint64_t seed, int in_order,
                                   uint16_t *__restrict__ Xb, float *__restrict__ yb) {
  const uint32_t i = blockIdx.x;
  if (i >= batch) return;
  uint64_t src = i;
  if (!in_order) {
    const U4 o = philox10(i, step, 0x4D4C5000u, 0u, (uint32_t)seed, (uint32_t)(seed >> 32));
    src = (((uint64_t)o.w[1] << 32) | o.w[0]) % n;
  }
  for (uint32_t c = threadIdx.x; c < width; c += blockDim.x) Xb[(uint64_t)i * width + c] = X[src * width + c];
  if (threadIdx.x == 0) yb[i] = y[src];
}

// ------------------------------------------------------------ term model

__device__ inline uint64_t frag_index(const LearnedDev *__restrict__ L, uint32_t f, uint64_t P) {
  uint64_t p = 0;
  for (uint32_t j = 0; j < L->n_axes[f]; ++j) p |= ((P >> (2 * L->axis_cut[f][j])) & 3ull) << (2 * j);
  return p;
}

// n_f[p] = sqrt(sum_b T_f[p][b]^2), rows summed in order
__global__ void colnorm_kernel(const double *__restrict__ T, uint32_t rows, uint64_t ncols,
                               double *__restrict__ out) {
  const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= ncols) return;
  double s = 0.0;
  for (uint32_t b = 0; b < rows; ++b) {
    const double t = T[p * rows + b];
    s += t * t;
  }
  out[p] = sqrt(s);
}

// The same for up to 64 rows per column: a wave stages 64 whole columns
// (contiguous in memory) through LDS with coalesced loads, all issued before
// the first store, then each lane sums its column in row order as above.
__global__ __launch_bounds__(64) void colnorm_tile_kernel(const double *__restrict__ T, uint32_t rows, uint64_t ncols,
                                                          double *__restrict__ out) {
  __shared__ double tile[64 * 65];  // column c at c * 65 (padded against bank conflicts)
  const uint64_t p0 = (uint64_t)blockIdx.x * 64;
  const uint32_t lane = threadIdx.x;
  const uint64_t cols = ncols - p0 < 64 ? ncols - p0 : 64;
  const uint32_t n = (uint32_t)(cols * rows);  // <= 4096 doubles
  const double *src = T + p0 * rows;
  for (uint32_t i0 = 0; i0 < n; i0 += 64 * 16) {
    double v[16];
#pragma unroll
    for (uint32_t k = 0; k < 16; ++k) {
      const uint32_t i = i0 + 64 * k + lane;
      v[k] = i < n ? src[i] : 0.0;
    }
#pragma unroll
    for (uint32_t k = 0; k < 16; ++k) {
      const uint32_t i = i0 + 64 * k + lane;
      if (i < n) tile[(i / rows) * 65 + i % rows] = v[k];
    }
  }
  __syncthreads();
  if (lane < cols) {
    double s = 0.0;
    for (uint32_t b = 0; b < rows; ++b) {
      const double t = tile[lane * 65 + b];
      s += t * t;
    }
    out[p0 + lane] = sqrt(s);
  }
}

// shares[j][d] = sum_{p: digit j of p = d} n[p]^2 / sum_p n[p]^2 for one
// fragment: slot 4 j + d sums the 4^(a-1) columns with that digit, in
// chunks (partials in order, then a fixed-order tree), then the chunks in
// order.
constexpr uint32_t kShareChunk = 4096;
__global__ __launch_bounds__(256) void share_partial_kernel(const double *__restrict__ norm, uint64_t per_slot,
                                                            uint32_t chunks, double *__restrict__ part) {
  __shared__ double red[256];
  const uint32_t slot = blockIdx.y, chunk = blockIdx.x;
  const uint32_t j = slot >> 2, d = slot & 3;
  const uint64_t low = (1ull << (2 * j)) - 1;
  const uint64_t e0 = (uint64_t)chunk * kShareChunk;
  const uint64_t e1 = e0 + kShareChunk < per_slot ? e0 + kShareChunk : per_slot;
  double acc = 0.0;
  for (uint64_t e = e0 + threadIdx.x; e < e1; e += 256) {
    const uint64_t p = ((e & ~low) << 2) | ((uint64_t)d << (2 * j)) | (e & low);
    acc += norm[p] * norm[p];
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (uint32_t w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(uint64_t)slot * chunks + chunk] = red[0];
}
__global__ void share_final_kernel(const double *__restrict__ part, uint32_t n_slots, uint32_t chunks,
                                   double *__restrict__ shares) {
  __shared__ double tot[4 * kMaxAxes];
  const uint32_t slot = threadIdx.x;
  if (slot < n_slots) {
    double sum = 0.0;
    for (uint32_t c = 0; c < chunks; ++c) sum += part[(uint64_t)slot * chunks + c];
    tot[slot] = sum;
  }
  __syncthreads();
  const double total = tot[0] + tot[1] + tot[2] + tot[3];
  if (slot < n_slots) shares[slot] = tot[slot] / total;
}

// phi tables of every cut: phi(s) = max(ln s, -40) / 40 of the share of the
// fragment on each side (src holds, per cut and side, the offset of that
// fragment's share row in `shares`, or -1 when the side has no fragment).
__global__ void phi_kernel(const double *__restrict__ shares, const int64_t *__restrict__ src, uint32_t k,
                           double *__restrict__ phi) {
  const uint32_t i = threadIdx.x;  // i = (c * 2 + side) * 4 + d
  if (i >= 8 * k) return;
  const uint32_t cs = i >> 2, d = i & 3;
  const int64_t o = src[cs];
  const double s = o < 0 ? 0.0 : shares[o + d];
  phi[i] = (s > 0.0 ? fmax(log(s), -40.0) : -40.0) / 40.0;
}

// Feature rows: columns 6c..6c+3 one-hot of P_c, 6c+4 phi_up(c, P_c),
// 6c+5 phi_dn(c, P_c), the rest zero (bf16).
__global__ void features_kernel(const LearnedDev *__restrict__ L, const uint64_t *__restrict__ terms,
                                uint64_t first, uint64_t n, uint32_t width, uint16_t *__restrict__ X) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * width) return;
  const uint64_t t = i / width;
  const uint32_t col = (uint32_t)(i % width);
  const uint64_t P = terms ? terms[t] : first + t;
  const uint32_t c = col / 6, r = col % 6;
  float v = 0.f;
  if (c < L->k) {
    const uint32_t p = (uint32_t)((P >> (2 * c)) & 3u);
    if (r < 4)
      v = r == p ? 1.f : 0.f;
    else
      v = (float)L->phi[(c * 2 + (r - 4)) * 4 + p];
  }
  X[i] = f2bf(v);
}

// Fused forward pass: a workgroup of 8 waves takes 128 term rows.  The
// rows' features are built in LDS (as features_kernel does); each layer's
// weights stream through LDS in chunks of 64 input columns; wave w
// accumulates rows 64 (w & 1) .. + 63 by columns 64 (w >> 1) .. + 63 with
// v_mfma_f32_16x16x16_bf16 in increasing k, adds the bias, applies the
// ReLU and rounds to bf16 into the activation tile (in place, after a
// barrier); the head then sums each row as head_forward_kernel does.
constexpr uint32_t FF_TM = 128, FF_H = 256, FF_F = 64, FF_KC = 64, FF_THREADS = 512;
constexpr uint32_t FF_AS = FF_H + 8, FF_WS = FF_KC + 8;  // padded row strides (bf16)

__device__ __attribute__((always_inline)) inline void ff_layer(uint16_t *act, uint16_t *ws, const uint16_t *__restrict__ W, const float *__restrict__ b,
                                uint32_t K, uint32_t tid) {
  const uint32_t lane = tid & 63, wave = tid >> 6;
  const uint32_t wm = (wave & 1) * 64, wn = (wave >> 1) * 64;
  float4v acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = float4v{0.f, 0.f, 0.f, 0.f};
  for (uint32_t kc = 0; kc < K; kc += FF_KC) {
    // weight chunk: ws[n][kk] = W[n][kc + kk], 256 rows of 128 B, four 16 B loads per thread
    u32x4 v0, v1, v2, v3;
    {
      const uint32_t i0 = tid, i1 = tid + FF_THREADS, i2 = tid + 2 * FF_THREADS, i3 = tid + 3 * FF_THREADS;
      v0 = *(const u32x4 *)(W + (uint64_t)(i0 >> 3) * K + kc + (i0 & 7) * 8);
      v1 = *(const u32x4 *)(W + (uint64_t)(i1 >> 3) * K + kc + (i1 & 7) * 8);
      v2 = *(const u32x4 *)(W + (uint64_t)(i2 >> 3) * K + kc + (i2 & 7) * 8);
      v3 = *(const u32x4 *)(W + (uint64_t)(i3 >> 3) * K + kc + (i3 & 7) * 8);
      __syncthreads();  // the previous chunk is consumed
      *(u32x4 *)&ws[(i0 >> 3) * FF_WS + (i0 & 7) * 8] = v0;
      *(u32x4 *)&ws[(i1 >> 3) * FF_WS + (i1 & 7) * 8] = v1;
      *(u32x4 *)&ws[(i2 >> 3) * FF_WS + (i2 & 7) * 8] = v2;
      *(u32x4 *)&ws[(i3 >> 3) * FF_WS + (i3 & 7) * 8] = v3;
    }
    __syncthreads();
#pragma unroll
    for (uint32_t ks = 0; ks < FF_KC; ks += 16) {
      short4v a[4], bb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        a[i] = *(const short4v *)&act[(wm + 16 * i + (lane & 15)) * FF_AS + kc + ks + 4 * (lane >> 4)];
#pragma unroll
      for (int j = 0; j < 4; ++j) bb[j] = *(const short4v *)&ws[(wn + 16 * j + (lane & 15)) * FF_WS + ks + 4 * (lane >> 4)];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], bb[j], acc[i][j], 0, 0, 0);
    }
  }
  __syncthreads();  // every wave is done reading this layer's input
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint32_t m = wm + 16 * i + 4 * (lane >> 4) + r, n = wn + 16 * j + (lane & 15);
        act[m * FF_AS + n] = f2bf(fmaxf(acc[i][j][r] + b[n], 0.f));
      }
  __syncthreads();
}

__global__ __launch_bounds__(FF_THREADS) void mlp_fused_forward_kernel(const LearnedDev *__restrict__ L,
                                                                       const MlpFused net, uint64_t first, uint64_t n,
                                                                       float scale, float *__restrict__ y) {
  extern __shared__ uint16_t ff_smem[];
  uint16_t *act = ff_smem;                     // [FF_TM][FF_AS]
  uint16_t *ws = ff_smem + FF_TM * FF_AS;      // [FF_H][FF_WS]
  const uint32_t tid = threadIdx.x;
  const uint64_t r0 = (uint64_t)blockIdx.x * FF_TM;
  // features of rows r0 .. r0 + 127 (zero rows past n)
  for (uint32_t i = tid; i < FF_TM * FF_F; i += FF_THREADS) {
    const uint32_t t = i / FF_F, col = i % FF_F;
    float v = 0.f;
    if (r0 + t < n) {
      const uint64_t P = first + r0 + t;
      const uint32_t c = col / 6, rr = col % 6;
      if (c < L->k) {
        const uint32_t p = (uint32_t)((P >> (2 * c)) & 3u);
        v = rr < 4 ? (rr == p ? 1.f : 0.f) : (float)L->phi[(c * 2 + (rr - 4)) * 4 + p];
      }
    }
    act[t * FF_AS + col] = f2bf(v);
  }
  __syncthreads();
  ff_layer(act, ws, net.w1, net.b1, FF_F, tid);
  ff_layer(act, ws, net.w2, net.b2, FF_H, tid);
  ff_layer(act, ws, net.w3, net.b3, FF_H, tid);
  // head: 32 lanes per row, eight consecutive elements per lane, butterfly
  const uint32_t l = tid & 31;
  for (uint32_t t = tid >> 5; t < FF_TM; t += FF_THREADS / 32) {
    float sacc = 0.f;
#pragma unroll
    for (int e = 0; e < 8; ++e) sacc += bf2f(act[t * FF_AS + l * 8 + e]) * bf2f(net.w4[l * 8 + e]);
#pragma unroll
    for (int o = 16; o > 0; o >>= 1) sacc += __shfl_xor(sacc, o, 32);
    if (l == 0 && r0 + t < n) y[r0 + t] = scale * (sacc + net.b4[0]);
  }
}

// kind 0: labels y(P) = ln(2^-k prod_f n_f[P|f] + 2^-60) (fp64, stored
// fp32); kind 2: y(P) / kLabelScale, the network's regression target;
// kind 1: the product-of-shares log-weights sum_c 40 (phi_up + phi_dn).
__global__ void labels_kernel(const LearnedDev *__restrict__ L, const uint64_t *__restrict__ terms,
                              uint64_t first, uint64_t n, float *__restrict__ y, int kind) {
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const uint64_t P = terms ? terms[t] : first + t;
  if (kind == 1) {
    double s = 0.0;
    for (uint32_t c = 0; c < L->k; ++c) {
      const uint32_t p = (uint32_t)((P >> (2 * c)) & 3u);
      s += 40.0 * (L->phi[(c * 2) * 4 + p] + L->phi[(c * 2 + 1) * 4 + p]);
    }
    y[t] = (float)s;
    return;
  }
  double v = ldexp(1.0, -(int)L->k);
  for (uint32_t f = 0; f < L->n_frags; ++f) v *= L->norm[f][frag_index(L, f, P)];
  const double lab = log(v + ldexp(1.0, -60));
  y[t] = (float)(kind == 2 ? lab / kLabelScale : lab);
}

// flags[P] = 1 if every fragment column of P has a nonzero norm
__global__ void support_flags_kernel(const LearnedDev *__restrict__ L, uint64_t K, uint64_t *__restrict__ flags) {
  const uint64_t P = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (P >= K) return;
  uint64_t ok = 1;
  for (uint32_t f = 0; f < L->n_frags; ++f) ok &= L->norm[f][frag_index(L, f, P)] > 0.0 ? 1u : 0u;
  flags[P] = ok;
}
// out[pos - 1] = P for flagged P, pos = inclusive prefix count
__global__ void support_scatter_kernel(const uint64_t *__restrict__ flags, const uint64_t *__restrict__ pos,
                                       uint64_t K, uint64_t cap, uint64_t *__restrict__ out) {
  const uint64_t P = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (P >= K || !flags[P]) return;
  if (pos[P] - 1 < cap) out[pos[P] - 1] = P;
}

// ------------------------------------------------------------ proposal

constexpr uint32_t kRedBlock = 256;
// stats[0] = max of the logits, stats[1] = sum exp(x - max) (fp64), each
// from per-block partials reduced in a fixed order.
__global__ void max_partial_kernel(const float *__restrict__ x, uint64_t n, float *__restrict__ part) {
  __shared__ float red[kRedBlock];
  float m = -INFINITY;
  for (uint64_t i = (uint64_t)blockIdx.x * kRedBlock + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kRedBlock)
    m = fmaxf(m, x[i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (uint32_t w = kRedBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}
// final reductions: thread t takes partials t, t + 256, ... in order, then a
// fixed tree over the 256 threads (deterministic)
__global__ __launch_bounds__(kRedBlock) void max_final_kernel(const float *__restrict__ part, uint32_t np,
                                                              double *__restrict__ stats) {
  __shared__ float red[kRedBlock];
  float m = -INFINITY;
  for (uint32_t i = threadIdx.x; i < np; i += kRedBlock) m = fmaxf(m, part[i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (uint32_t w = kRedBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) stats[0] = (double)red[0];
}
__global__ void sumexp_partial_kernel(const float *__restrict__ x, uint64_t n, const double *__restrict__ stats,
                                      double *__restrict__ part) {
  __shared__ double red[kRedBlock];
  const double mx = stats[0];
  double s = 0.0;
  for (uint64_t i = (uint64_t)blockIdx.x * kRedBlock + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kRedBlock)
    s += exp((double)x[i] - mx);
  red[threadIdx.x] = s;
  __syncthreads();
  for (uint32_t w = kRedBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}
__global__ __launch_bounds__(kRedBlock) void sum_final_kernel(const double *__restrict__ part, uint32_t np,
                                                              double *__restrict__ stats) {
  __shared__ double red[kRedBlock];
  double s = 0.0;
  for (uint32_t i = threadIdx.x; i < np; i += kRedBlock) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (uint32_t w = kRedBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) stats[1] = red[0];
}
// q = (1 - eps) exp(x - max) / S + eps / n; uniform 1 / n without logits
__global__ void proposal_kernel(const float *__restrict__ x, uint64_t n, const double *__restrict__ stats, double eps,
                                double *__restrict__ q) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (!x) {
    q[i] = 1.0 / (double)n;
    return;
  }
  q[i] = (1.0 - eps) * exp((double)x[i] - stats[0]) / stats[1] + eps / (double)n;
}

// integer weights floor(q 2^40)
__global__ void int_weights_kernel(const double *__restrict__ q, uint64_t n, uint64_t *__restrict__ w) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) w[i] = (uint64_t)floor(q[i] * 1099511627776.0);
}

// Inclusive scan of u64 in blocks of 1024 (four per thread), block totals
// out; a second level scans the totals and a third adds them back.
constexpr uint32_t kScanBlock = 256, kScanPer = 4, kScanTile = kScanBlock * kScanPer;
__global__ __launch_bounds__(kScanBlock) void scan_tile_kernel(uint64_t *__restrict__ x, uint64_t n,
                                                               uint64_t *__restrict__ totals) {
  __shared__ uint64_t s[kScanBlock];
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile + threadIdx.x * kScanPer;
  uint64_t v[kScanPer];
  uint64_t run = 0;
#pragma unroll
  for (uint32_t i = 0; i < kScanPer; ++i) {
    run += base + i < n ? x[base + i] : 0;
    v[i] = run;
  }
  s[threadIdx.x] = run;
  __syncthreads();
  for (uint32_t o = 1; o < kScanBlock; o <<= 1) {
    const uint64_t add = threadIdx.x >= o ? s[threadIdx.x - o] : 0;
    __syncthreads();
    s[threadIdx.x] += add;
    __syncthreads();
  }
  const uint64_t before = threadIdx.x ? s[threadIdx.x - 1] : 0;
#pragma unroll
  for (uint32_t i = 0; i < kScanPer; ++i)
    if (base + i < n) x[base + i] = v[i] + before;
  if (threadIdx.x == kScanBlock - 1 && totals) totals[blockIdx.x] = s[kScanBlock - 1];
}
__global__ void scan_add_kernel(uint64_t *__restrict__ x, uint64_t n, const uint64_t *__restrict__ scanned_totals) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t tile = i / kScanTile;
  if (i < n && tile > 0) x[i] += scanned_totals[tile - 1];
}

// Term j: u = (o1 2^32 + o0) mod C[K-1] from Philox(ctr = (j, 0, lo cid,
// hi cid), key = (lo seed ^ 0x7E570001, hi seed)); the term is the smallest
// P with C[P] > u.
__global__ void sample_terms_kernel(const uint64_t *__restrict__ cdf, uint64_t K, uint64_t n, uint64_t seed,
                                    uint64_t cid, uint64_t *__restrict__ out) {
  const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const U4 o = philox10((uint32_t)j, 0u, (uint32_t)cid, (uint32_t)(cid >> 32), (uint32_t)seed ^ 0x7E570001u,
                        (uint32_t)(seed >> 32));
  const uint64_t total = cdf[K - 1];
  if (total == 0) {  // every integer weight rounded to zero: no valid draw
    out[j] = 0;
    return;
  }
  const uint64_t u = (((uint64_t)o.w[1] << 32) | o.w[0]) % total;
  uint64_t lo = 0, hi = K - 1;  // cdf[hi] = total > u
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    if (cdf[mid] > u)
      hi = mid;
    else
      lo = mid + 1;
  }
  out[j] = lo;
}

// importance weights 1 / (N q[P_j])
__global__ void is_scale_kernel(const uint64_t *__restrict__ terms, const double *__restrict__ q, uint64_t n,
                                double *__restrict__ scale) {
  const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) scale[j] = 1.0 / ((double)n * q[terms[j]]);
}

inline unsigned blocks(uint64_t n, uint32_t b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t launch_mlp_gemm(const MlpGemm &g, int epi, hipStream_t s) {
  if (g.N % MG_T || g.K % MG_K || (g.sak != 1 && g.sam != 1) || (g.sbk != 1 && g.sbn != 1))
    return hipErrorInvalidValue;
  const uint64_t tm = (g.M + MG_T - 1) / MG_T;
  if (tm == 0) return hipSuccess;
  if (tm > 0x7FFFFFFFull) return hipErrorInvalidValue;
  const dim3 grid((unsigned)tm, g.N / MG_T);
  switch (epi) {
    case MLP_EPI_F32: hipLaunchKernelGGL(mlp_gemm_kernel<MLP_EPI_F32>, grid, dim3(MG_THREADS), 0, s, g); break;
    case MLP_EPI_BIAS_RELU:
      hipLaunchKernelGGL(mlp_gemm_kernel<MLP_EPI_BIAS_RELU>, grid, dim3(MG_THREADS), 0, s, g);
      break;
    case MLP_EPI_MASK: hipLaunchKernelGGL(mlp_gemm_kernel<MLP_EPI_MASK>, grid, dim3(MG_THREADS), 0, s, g); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_mlp_logits_fused(const LearnedDev *L, const MlpFused &net, uint64_t first, uint64_t n, float scale,
                                   float *y, hipStream_t s) {
  if (net.F != FF_F || net.H != FF_H) return hipErrorInvalidValue;
  if (n == 0) return hipSuccess;
  const size_t lds = (size_t)(FF_TM * FF_AS + FF_H * FF_WS) * sizeof(uint16_t);
  hipError_t e = hipFuncSetAttribute((const void *)mlp_fused_forward_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const uint64_t blocks_n = (n + FF_TM - 1) / FF_TM;
  if (blocks_n > 0x7FFFFFFFull) return hipErrorInvalidValue;
  hipLaunchKernelGGL(mlp_fused_forward_kernel, dim3((unsigned)blocks_n), dim3(FF_THREADS), lds, s, L, net, first, n,
                     scale, y);
  return hipGetLastError();
}

hipError_t launch_head_forward(const uint16_t *H, uint32_t width, uint64_t rows, const uint16_t *w, const float *b,
                               float scale, float *y, hipStream_t s) {
  if (width % 8 || rows == 0) return rows == 0 ? hipSuccess : hipErrorInvalidValue;
  hipLaunchKernelGGL(head_forward_kernel, dim3(blocks(rows * 32, 256)), dim3(256), 0, s, H, width, rows, w, b, scale,
                     y);
  return hipGetLastError();
}

hipError_t launch_head_backward(const uint16_t *H, uint32_t width, uint64_t rows, const uint16_t *w, const float *y,
                                const float *t, float *dy, float *sq, uint16_t *dZ, hipStream_t s) {
  hipLaunchKernelGGL(head_backward_kernel, dim3(blocks(rows * width, 256)), dim3(256), 0, s, H, width, rows, w, y, t,
                     2.0f / (float)rows, dy, sq, dZ);
  return hipGetLastError();
}

uint32_t colsum_chunks(uint64_t rows) { return (uint32_t)((rows + kColChunk - 1) / kColChunk); }

hipError_t launch_colsum(const uint16_t *X, uint32_t width, uint64_t rows, const float *sc, float *part, float *out,
                         hipStream_t s) {
  if (width > 256) return hipErrorInvalidValue;
  const uint32_t ch = colsum_chunks(rows);
  hipLaunchKernelGGL(colsum_partial_kernel, dim3(ch), dim3(256), 0, s, X, width, rows, sc, part);
  hipLaunchKernelGGL(colsum_final_kernel, dim3(blocks(width, 256)), dim3(256), 0, s, part, width, ch, out);
  return hipGetLastError();
}

hipError_t launch_vsum(const float *x, uint64_t n, float *out, hipStream_t s) {
  hipLaunchKernelGGL(vsum_kernel, dim3(1), dim3(256), 0, s, x, n, out);
  return hipGetLastError();
}

hipError_t launch_adam(float *p, const float *g, float *m, float *v, uint16_t *pb, uint64_t n, float lr, float b1,
                       float b2, float c1, float c2, float eps, hipStream_t s) {
  hipLaunchKernelGGL(adam_kernel, dim3(blocks(n, 256)), dim3(256), 0, s, p, g, m, v, pb, n, lr, b1, b2, c1, c2, eps);
  return hipGetLastError();
}

hipError_t launch_to_bf16(const float *p, uint16_t *pb, uint64_t n, hipStream_t s) {
  hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks(n, 256)), dim3(256), 0, s, p, pb, n);
  return hipGetLastError();
}

hipError_t launch_gather_rows(const uint16_t *X, const float *y, uint64_t n, uint32_t width, uint32_t batch,
                              uint32_t step, uint64_t seed, int in_order, uint16_t *Xb, float *yb, hipStream_t s) {
  hipLaunchKernelGGL(gather_rows_kernel, dim3(batch), dim3(64), 0, s, X, y, n, width, batch, step, seed, in_order, Xb,
                     yb);
  return hipGetLastError();
}

hipError_t launch_colnorm(const double *T, uint32_t rows, uint64_t ncols, double *out, hipStream_t s) {
  if (rows <= 64)
    hipLaunchKernelGGL(colnorm_tile_kernel, dim3(blocks(ncols, 64)), dim3(64), 0, s, T, rows, ncols, out);
  else
    hipLaunchKernelGGL(colnorm_kernel, dim3(blocks(ncols, 256)), dim3(256), 0, s, T, rows, ncols, out);
  return hipGetLastError();
}

hipError_t launch_shares(const double *norm, uint32_t n_axes, double *part, double *shares, hipStream_t s) {
  if (n_axes == 0) return hipSuccess;
  if (n_axes > (uint32_t)kMaxAxes) return hipErrorInvalidValue;
  const uint64_t per_slot = 1ull << (2 * (n_axes - 1));
  const uint32_t chunks = share_chunks(n_axes);
  hipLaunchKernelGGL(share_partial_kernel, dim3(chunks, 4 * n_axes), dim3(256), 0, s, norm, per_slot, chunks, part);
  hipLaunchKernelGGL(share_final_kernel, dim3(1), dim3(4 * kMaxAxes), 0, s, part, 4 * n_axes, chunks, shares);
  return hipGetLastError();
}

uint32_t share_chunks(uint32_t n_axes) {
  if (n_axes == 0) return 1;
  const uint64_t per_slot = 1ull << (2 * (n_axes - 1));
  return (uint32_t)((per_slot + kShareChunk - 1) / kShareChunk);
}

hipError_t launch_phi(const double *shares, const int64_t *src, uint32_t k, double *phi, hipStream_t s) {
  if (8 * k > 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL(phi_kernel, dim3(1), dim3(8 * k), 0, s, shares, src, k, phi);
  return hipGetLastError();
}

hipError_t launch_features(const LearnedDev *L, const uint64_t *terms, uint64_t first, uint64_t n, uint32_t width,
                           uint16_t *X, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(features_kernel, dim3(blocks(n * width, 256)), dim3(256), 0, s, L, terms, first, n, width, X);
  return hipGetLastError();
}

hipError_t launch_labels(const LearnedDev *L, const uint64_t *terms, uint64_t first, uint64_t n, float *y, int kind,
                         hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(labels_kernel, dim3(blocks(n, 256)), dim3(256), 0, s, L, terms, first, n, y, kind);
  return hipGetLastError();
}

hipError_t launch_support(const LearnedDev *L, uint64_t K, uint64_t *flags, uint64_t *pos, uint64_t *scratch,
                          uint64_t cap, uint64_t *out, hipStream_t s) {
  hipLaunchKernelGGL(support_flags_kernel, dim3(blocks(K, 256)), dim3(256), 0, s, L, K, flags);
  hipError_t e = hipMemcpyAsync(pos, flags, K * 8, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return e;
  if ((e = launch_scan_u64(pos, K, scratch, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(support_scatter_kernel, dim3(blocks(K, 256)), dim3(256), 0, s, flags, pos, K, cap, out);
  return hipGetLastError();
}

uint64_t scan_scratch_words(uint64_t n) {
  uint64_t w = 0;
  while (n > kScanTile) {
    n = (n + kScanTile - 1) / kScanTile;
    w += n;
  }
  return w + 1;
}

hipError_t launch_scan_u64(uint64_t *x, uint64_t n, uint64_t *scratch, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const uint64_t tiles = (n + kScanTile - 1) / kScanTile;
  if (tiles > 0x7FFFFFFFull) return hipErrorInvalidValue;
  if (tiles == 1) {
    hipLaunchKernelGGL(scan_tile_kernel, dim3(1), dim3(kScanBlock), 0, s, x, n, (uint64_t *)nullptr);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(scan_tile_kernel, dim3((unsigned)tiles), dim3(kScanBlock), 0, s, x, n, scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = launch_scan_u64(scratch, tiles, scratch + tiles, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(scan_add_kernel, dim3(blocks(n, 256)), dim3(256), 0, s, x, n, scratch);
  return hipGetLastError();
}

uint32_t reduce_blocks(uint64_t n) {
  const uint64_t b = (n + kRedBlock - 1) / kRedBlock;
  return (uint32_t)(b < 1024 ? (b ? b : 1) : 1024);
}

hipError_t launch_proposal(const float *logits, uint64_t n, double eps, float *mpart, double *spart, double *stats,
                           double *q, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const uint32_t nb = reduce_blocks(n);
  if (logits) {
    hipLaunchKernelGGL(max_partial_kernel, dim3(nb), dim3(kRedBlock), 0, s, logits, n, mpart);
    hipLaunchKernelGGL(max_final_kernel, dim3(1), dim3(kRedBlock), 0, s, mpart, nb, stats);
    hipLaunchKernelGGL(sumexp_partial_kernel, dim3(nb), dim3(kRedBlock), 0, s, logits, n, stats, spart);
    hipLaunchKernelGGL(sum_final_kernel, dim3(1), dim3(kRedBlock), 0, s, spart, nb, stats);
  }
  hipLaunchKernelGGL(proposal_kernel, dim3(blocks(n, 256)), dim3(256), 0, s, logits, n, stats, eps, q);
  return hipGetLastError();
}

hipError_t launch_int_cdf(const double *q, uint64_t n, uint64_t *cdf, uint64_t *scratch, hipStream_t s) {
  hipLaunchKernelGGL(int_weights_kernel, dim3(blocks(n, 256)), dim3(256), 0, s, q, n, cdf);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_scan_u64(cdf, n, scratch, s);
}

hipError_t launch_sample_terms(const uint64_t *cdf, uint64_t K, uint64_t n, uint64_t seed, uint64_t cid,
                               uint64_t *out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(sample_terms_kernel, dim3(blocks(n, 256)), dim3(256), 0, s, cdf, K, n, seed, cid, out);
  return hipGetLastError();
}

hipError_t launch_is_scale(const uint64_t *terms, const double *q, uint64_t n, double *scale, hipStream_t s) {
  hipLaunchKernelGGL(is_scale_kernel, dim3(blocks(n, 256)), dim3(256), 0, s, terms, q, n, scale);
  return hipGetLastError();
}

}  // namespace ccut

// ------------------------------------------------ term draws without allocation
// ccut_sample_terms_noalloc keeps the integer CDF and the scan partials of a
// draw in one fixed device array instead of allocating them: up to
// kNoAllocMaxTerms cut terms (4^10, the ten-cut recombination) plus the scan
// partials of that size, 8 MiB + 16 KiB on each device the library runs on,
// held until the process ends.  Host code never uses the array's name as an
// address: its device address is looked up once per device with
// hipGetSymbolAddress (with that device current) and kept.
namespace {

constexpr uint64_t kNoAllocMaxTerms = 1ull << 20;
constexpr uint64_t kNoAllocScanWords = 2048;  // scan partials for up to kNoAllocMaxTerms entries (1025 words)
constexpr uint64_t kNoAllocWords = kNoAllocMaxTerms + kNoAllocScanWords;
constexpr int kNoAllocMaxDevices = 64;

static __device__ __align__(256) uint64_t noalloc_scratch[kNoAllocWords];

std::mutex g_noalloc_mu;
uint64_t *g_noalloc_ptr[kNoAllocMaxDevices] = {};

}  // namespace

extern "C" ccut_status ccut_sample_terms_noalloc(void *hip_stream, const double *q, uint64_t K, uint64_t n,
                                                 uint64_t seed, uint64_t cid, uint64_t *out) {
  using namespace ccut;
  if (!q || K == 0 || (n && !out)) {
    set_call_error("ccut_sample_terms_noalloc: NULL argument or K = 0");
    return CCUT_E_INVALID;
  }
  if (n > 0xFFFFFFFFull) {
    set_call_error("ccut_sample_terms_noalloc: at most 2^32 - 1 terms per draw");
    return CCUT_E_INVALID;
  }
  if (K > kNoAllocMaxTerms || scan_scratch_words(K) > kNoAllocScanWords) {
    set_call_error("ccut_sample_terms_noalloc: K above 2^20, the size of the fixed term buffer");
    return CCUT_E_UNSUPPORTED;
  }
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kNoAllocMaxDevices) {
    set_call_error("ccut_sample_terms_noalloc: no current HIP device");
    return CCUT_E_DEVICE;
  }
  uint64_t *base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
      void *ptr = nullptr;
      if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(noalloc_scratch)) != hipSuccess || !ptr) {
        set_call_error("ccut_sample_terms_noalloc: hipGetSymbolAddress of the term buffer failed");
        return CCUT_E_DEVICE;
      }
      g_noalloc_ptr[dev] = static_cast<uint64_t *>(ptr);
    }
    base = g_noalloc_ptr[dev];
  }
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  // every CDF entry and scan partial is written before it is read: nothing
  // left by an earlier call is used
  uint64_t *cdf = base, *partials = base + K;
  if (launch_int_cdf(q, K, cdf, partials, s) != hipSuccess ||
      launch_sample_terms(cdf, K, n, seed, cid, out, s) != hipSuccess) {
    set_call_error("ccut_sample_terms_noalloc: kernel launch failed");
    return CCUT_E_DEVICE;
  }
  return CCUT_OK;
}

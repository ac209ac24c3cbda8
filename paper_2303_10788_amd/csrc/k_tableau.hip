// Clifford fragment variant -> affine sample model (x0, randmask, G).
//
// One workgroup evaluates one variant on a stabilizer tableau in the
// Aaronson-Gottesman layout (destabilizer rows 0..m-1, stabilizer rows
// m..2m-1), the tableau the paper's Clifford backend builds on
// (Sec. III-B).  Rows are bit-packed in uint64 words and stored word-major
// in LDS, X[w][row], Z[w][row], so the rows of one gate column are
// contiguous and a thread owns a fixed set of rows for the whole gate
// phase (no barrier between gates).
//
// Signs are carried symbolically.  A stabilizer's sign is an affine GF(2)
// form over the outcomes of the random measurements made so far:
// (constant bit, coefficient mask over measurement indices).  A random
// measurement's outcome is its own fresh bit, so after all measurements a
// shot is x = x0 ^ G u with u the per-measurement Philox bits.  Whether a
// measurement is random, and every x/z bit, never depends on earlier
// outcomes; the affine form is therefore exactly the per-shot tableau
// simulation with the same bits.
//
// Phases use the i^(x.z) form of a Hermitian Pauli: (-1)^r X^x Z^z carries
// phase exponent a = 2r + popc(x & z) (mod 4), and the product of
// P1 = i^a1 X^x1 Z^z1 and P2 = i^a2 X^x2 Z^z2 is
// i^(a1 + a2 + 2 popc(z1 & x2)) X^(x1^x2) Z^(z1^z2).
#include "common.hpp"

namespace ccut {

namespace {

template <int W>
struct RowAcc {
  uint64_t x[W];
  uint64_t z[W];
  uint64_t form;
  uint32_t num;  // phase exponent numerator, mod 4
};

template <int W>
__device__ inline void acc_combine(RowAcc<W> &L, const RowAcc<W> &R) {
  uint32_t cross = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) cross += __popcll(L.z[w] & R.x[w]);
  L.num = (L.num + R.num + 2u * cross) & 3u;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    L.x[w] ^= R.x[w];
    L.z[w] ^= R.z[w];
  }
  L.form ^= R.form;
}

template <int W>
__device__ inline RowAcc<W> acc_shfl_xor(const RowAcc<W> &a, int mask) {
  RowAcc<W> b;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    b.x[w] = __shfl_xor(a.x[w], mask);
    b.z[w] = __shfl_xor(a.z[w], mask);
  }
  b.form = __shfl_xor(a.form, mask);
  b.num = (uint32_t)__shfl_xor((int)a.num, mask);
  return b;
}

// Apply one Clifford gate to row i (stabilizer rows also update their sign
// constant; destabilizer signs never reach an outcome and are not kept).
template <int W>
__device__ inline void gate_row(uint64_t *X, uint64_t *Z, uint32_t *CST, int R2, int m, int i,
                                uint32_t kind, uint32_t a, uint32_t b) {
  const int wa = (int)(a >> 6);
  const uint64_t ma = 1ull << (a & 63);
  uint64_t *xa_p = X + wa * R2 + i;
  uint64_t *za_p = Z + wa * R2 + i;
  uint32_t flip = 0;
  switch (kind) {
    case G_H: {
      uint64_t x = *xa_p, z = *za_p;
      uint32_t xa = (x & ma) != 0, za = (z & ma) != 0;
      flip = xa & za;
      uint64_t d = (x ^ z) & ma;
      *xa_p = x ^ d;
      *za_p = z ^ d;
      break;
    }
    case G_S: {
      uint64_t x = *xa_p, z = *za_p;
      uint32_t xa = (x & ma) != 0, za = (z & ma) != 0;
      flip = xa & za;
      if (xa) *za_p = z ^ ma;
      break;
    }
    case G_SDG: {
      uint64_t x = *xa_p, z = *za_p;
      uint32_t xa = (x & ma) != 0, za = (z & ma) != 0;
      flip = xa & (za ^ 1u);
      if (xa) *za_p = z ^ ma;
      break;
    }
    case G_X:
      flip = (*za_p & ma) != 0;
      break;
    case G_Y:
      flip = ((*xa_p ^ *za_p) & ma) != 0;
      break;
    case G_Z:
      flip = (*xa_p & ma) != 0;
      break;
    case G_CX: {
      const int wb = (int)(b >> 6);
      const uint64_t mb = 1ull << (b & 63);
      uint64_t *xb_p = X + wb * R2 + i;
      uint64_t *zb_p = Z + wb * R2 + i;
      uint32_t xc = (*xa_p & ma) != 0, zc = (*za_p & ma) != 0;
      uint32_t xt = (*xb_p & mb) != 0, zt = (*zb_p & mb) != 0;
      flip = xc & zt & (xt ^ zc ^ 1u);
      if (xc) *xb_p ^= mb;
      if (zt) *za_p ^= ma;
      break;
    }
    case G_CZ: {
      const int wb = (int)(b >> 6);
      const uint64_t mb = 1ull << (b & 63);
      uint64_t *zb_p = Z + wb * R2 + i;
      uint32_t x1 = (*xa_p & ma) != 0, z1 = (*za_p & ma) != 0;
      uint32_t x2 = (X[wb * R2 + i] & mb) != 0, z2 = (*zb_p & mb) != 0;
      flip = x1 & x2 & (z1 ^ z2);
      if (x2) *za_p ^= ma;
      if (x1) *zb_p ^= mb;
      break;
    }
    default:
      break;
  }
  if (i >= m) CST[i - m] ^= flip;
}

// LDS bytes for a width-m fragment with W words per row half.
template <int W, int BLOCK>
size_t tableau_lds(size_t m) {
  size_t b = (2 * W * 2 * m + m + 64 + 1) * 8;    // X, Z, FORM, GROW, X0
  b += (BLOCK / 64) * sizeof(RowAcc<W>);         // RED
  b += m * 4 + 8;                                // CST, PIV
  return (b + 15) & ~size_t(15);
}

template <int W, int BLOCK>
__global__ __launch_bounds__(BLOCK) void tableau_kernel(const FragDev *__restrict__ fd, uint64_t v0,
                                                        uint64_t *__restrict__ models) {
  extern __shared__ uint64_t smem[];
  const FragDev &F = *fd;
  const int m = (int)F.m;
  const int R2 = 2 * m;
  const int tid = threadIdx.x;
  const uint64_t v = v0 + blockIdx.x;
  const uint32_t n_meas = F.n_meas;

  uint64_t *X = smem;                    // [W][2m]
  uint64_t *Z = X + (size_t)W * R2;      // [W][2m]
  uint64_t *FORM = Z + (size_t)W * R2;   // [m] stabilizer sign forms
  uint64_t *GROW = FORM + m;             // [64] outcome forms per measurement
  uint64_t *X0 = GROW + 64;              // [1] deterministic outcome constants
  RowAcc<W> *RED = reinterpret_cast<RowAcc<W> *>(X0 + 1);  // [BLOCK/64]
  uint32_t *CST = reinterpret_cast<uint32_t *>(RED + BLOCK / 64);  // [m]
  int *PIV = reinterpret_cast<int *>(CST + m);

  for (int i = tid; i < R2; i += BLOCK) {
#pragma unroll
    for (int w = 0; w < W; ++w) {
      X[w * R2 + i] = (i < m && (i >> 6) == w) ? (1ull << (i & 63)) : 0ull;
      Z[w * R2 + i] = (i >= m && ((i - m) >> 6) == w) ? (1ull << ((i - m) & 63)) : 0ull;
    }
  }
  for (int i = tid; i < m; i += BLOCK) {
    FORM[i] = 0;
    CST[i] = 0;
  }
  if (tid < 64) GROW[tid] = 0;
  if (tid == 0) *X0 = 0;
  __syncthreads();

  // ---- gate phase: every thread updates only its own rows, so no barrier
  // is needed between gates.  Preparations on quantum inputs:
  // |0>, |1> = X|0>, |+> = H|0>, |+i> = S H|0>.
  {
    uint64_t t = v;
    for (uint32_t j = 0; j < F.n_axes; ++j) {
      const uint32_t d = (uint32_t)(t % F.axis_radix[j]);
      t /= F.axis_radix[j];
      if (F.axis_side[j] != 1 || d == 0) continue;
      const uint32_t q = F.axis_local[j];
      for (int i = tid; i < R2; i += BLOCK) {
        if (d == 1) {
          gate_row<W>(X, Z, CST, R2, m, i, G_X, q, 0);
        } else {
          gate_row<W>(X, Z, CST, R2, m, i, G_H, q, 0);
          if (d == 3) gate_row<W>(X, Z, CST, R2, m, i, G_S, q, 0);
        }
      }
    }
  }
  for (uint32_t g = 0; g < F.n_ops; ++g) {
    const uint32_t word = F.ops[g];
    const uint32_t kind = op_kind(word), a = op_q0(word), b = op_q1(word);
    for (int i = tid; i < R2; i += BLOCK) gate_row<W>(X, Z, CST, R2, m, i, kind, a, b);
  }
  // basis rotations on quantum outputs: X -> H, Y -> S^dag then H, Z -> none
  {
    uint64_t t = v;
    for (uint32_t j = 0; j < F.n_axes; ++j) {
      const uint32_t d = (uint32_t)(t % F.axis_radix[j]);
      t /= F.axis_radix[j];
      if (F.axis_side[j] != 0 || d == 2) continue;
      const uint32_t q = F.axis_local[j];
      for (int i = tid; i < R2; i += BLOCK) {
        if (d == 1) gate_row<W>(X, Z, CST, R2, m, i, G_SDG, q, 0);
        gate_row<W>(X, Z, CST, R2, m, i, G_H, q, 0);
      }
    }
  }
  __syncthreads();

  // ---- measurements of the measured set, in order
  uint64_t randmask = 0;
  for (uint32_t j = 0; j < n_meas; ++j) {
    const uint32_t a = F.meas[j];
    const int wa = (int)(a >> 6);
    const uint64_t ma = 1ull << (a & 63);
    if (tid == 0) PIV[0] = 0x7FFFFFFF;
    __syncthreads();
    int lmin = 0x7FFFFFFF;
    for (int i = m + tid; i < R2; i += BLOCK)
      if (X[wa * R2 + i] & ma) {
        lmin = i;
        break;
      }
    if (lmin != 0x7FFFFFFF) atomicMin(&PIV[0], lmin);
    __syncthreads();
    const int p = PIV[0];
    if (p != 0x7FFFFFFF) {
      // random outcome: multiply row p into every other row with x_a = 1
      uint64_t xp[W], zp[W];
      uint32_t pc_p = 0;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        xp[w] = X[w * R2 + p];
        zp[w] = Z[w * R2 + p];
        pc_p += __popcll(xp[w] & zp[w]);
      }
      const uint64_t formp = FORM[p - m];
      const uint32_t cstp = CST[p - m];
      for (int i = tid; i < R2; i += BLOCK) {
        if (i == p || !(X[wa * R2 + i] & ma)) continue;
        uint32_t c2 = 0, c3 = 0, c4 = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) {
          const uint64_t xi = X[w * R2 + i], zi = Z[w * R2 + i];
          c2 += __popcll(xi & zi);
          c3 += __popcll(zp[w] & xi);
          const uint64_t xn = xi ^ xp[w], zn = zi ^ zp[w];
          c4 += __popcll(xn & zn);
          X[w * R2 + i] = xn;
          Z[w * R2 + i] = zn;
        }
        if (i >= m) {
          const uint32_t num = 2u * cstp + pc_p + 2u * CST[i - m] + c2 + 2u * c3 - c4;
          CST[i - m] = (num & 3u) >> 1;
          FORM[i - m] ^= formp;
        }
      }
      __syncthreads();
      if (tid == 0) {
#pragma unroll
        for (int w = 0; w < W; ++w) {
          X[w * R2 + (p - m)] = xp[w];
          Z[w * R2 + (p - m)] = zp[w];
          X[w * R2 + p] = 0;
          Z[w * R2 + p] = (w == wa) ? ma : 0ull;
        }
        FORM[p - m] = 1ull << j;
        CST[p - m] = 0;
        GROW[j] = 1ull << j;
      }
      randmask |= 1ull << j;
      __syncthreads();
    } else {
      // deterministic: the outcome is the sign of the product of the
      // stabilizers paired with destabilizers that have x_a = 1
      RowAcc<W> acc;
#pragma unroll
      for (int w = 0; w < W; ++w) acc.x[w] = acc.z[w] = 0;
      acc.form = 0;
      acc.num = 0;
      for (int i = tid; i < m; i += BLOCK) {
        if (!(X[wa * R2 + i] & ma)) continue;
        RowAcc<W> r;
        uint32_t pc = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) {
          r.x[w] = X[w * R2 + m + i];
          r.z[w] = Z[w * R2 + m + i];
          pc += __popcll(r.x[w] & r.z[w]);
        }
        r.form = FORM[i];
        r.num = (2u * CST[i] + pc) & 3u;
        acc_combine<W>(acc, r);
      }
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        RowAcc<W> o = acc_shfl_xor<W>(acc, off);
        if ((tid & off) == 0) {
          acc_combine<W>(acc, o);
        } else {
          acc_combine<W>(o, acc);
          acc = o;
        }
      }
      if ((tid & 63) == 0) RED[tid >> 6] = acc;
      __syncthreads();
      if (tid == 0) {
        RowAcc<W> tot = RED[0];
        for (int wv = 1; wv < BLOCK / 64; ++wv) acc_combine<W>(tot, RED[wv]);
        // tot is +-Z_a: x = 0, z = e_a, so its sign bit is num / 2
        *X0 |= (uint64_t)((tot.num & 3u) >> 1) << j;
        GROW[j] = tot.form;
      }
      __syncthreads();
    }
  }

  // ---- write the model: x0, randmask, and G by columns
  uint64_t *out = models + (size_t)blockIdx.x * model_words(n_meas);
  if (tid == 0) {
    out[0] = *X0;
    out[1] = randmask;
  }
  for (uint32_t c = tid; c < n_meas; c += BLOCK) {
    uint64_t col = 0;
    for (uint32_t j = 0; j < n_meas; ++j) col |= ((GROW[j] >> c) & 1ull) << j;
    out[2 + c] = col;
  }
}

template <int W, int BLOCK>
hipError_t launch_w(const FragDev *d_frag, const FragDev &h, uint64_t v0, uint64_t nv,
                    uint64_t *models, hipStream_t s) {
  const size_t lds = tableau_lds<W, BLOCK>(h.m);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute((const void *)tableau_kernel<W, BLOCK>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  for (uint64_t done = 0; done < nv;) {
    uint64_t chunk = nv - done;
    if (chunk > (1ull << 30)) chunk = 1ull << 30;
    hipLaunchKernelGGL((tableau_kernel<W, BLOCK>), dim3((unsigned)chunk), dim3(BLOCK), lds, s, d_frag,
                       v0 + done, models + done * model_words(h.n_meas));
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    done += chunk;
  }
  return hipSuccess;
}

}  // namespace

hipError_t launch_tableau(const FragDev *d_frag, const FragDev &h, uint64_t v0, uint64_t nv,
                          uint64_t *models, hipStream_t s) {
  if (h.n_meas > (uint32_t)kMaxMeas) return hipErrorInvalidValue;
  const uint32_t W = (h.m + 63) / 64;
  if (W <= 1) return launch_w<1, 64>(d_frag, h, v0, nv, models, s);
  if (W <= 2) return launch_w<2, 128>(d_frag, h, v0, nv, models, s);
  if (W <= 4) return launch_w<4, 256>(d_frag, h, v0, nv, models, s);
  if (W <= 8) return launch_w<8, 256>(d_frag, h, v0, nv, models, s);
  return hipErrorInvalidValue;
}

}  // namespace ccut

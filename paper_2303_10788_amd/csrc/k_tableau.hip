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
#include <algorithm>
#include <type_traits>

#include "common.hpp"

namespace ccut {

namespace {

// Preparation of a quantum input (digit d: |0>, |1> = X|0>, |+> = H|0>,
// |+i> = S H|0>) and basis rotation of a quantum output (digit d: X -> H,
// Y -> S^dag then H, Z -> none) as one-qubit Clifford maps.
__device__ inline uint32_t prep_c1(uint32_t d) {
  return d == 1 ? c1_of_gate(G_X) : d == 2 ? c1_of_gate(G_H) : d == 3 ? c1_then(c1_of_gate(G_H), c1_of_gate(G_S)) : 0u;
}
__device__ inline uint32_t basis_c1(uint32_t d) {
  return d == 0 ? c1_of_gate(G_H) : d == 1 ? c1_then(c1_of_gate(G_SDG), c1_of_gate(G_H)) : 0u;
}

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
// constant; destabilizer signs never reach an outcome and are not kept):
// CX, CZ, or a fused one-qubit Clifford (G_C1 parameters in b).
template <int W>
__device__ inline void gate_row(uint64_t *X, uint64_t *Z, uint32_t *CST, int R2, int m, int i,
                                uint32_t kind, uint32_t a, uint32_t b) {
  const int wa = (int)(a >> 6);
  const uint32_t sa = a & 63;
  uint64_t *xa_p = X + wa * R2 + i;
  uint64_t *za_p = Z + wa * R2 + i;
  uint32_t flip = 0;
  if (kind == G_CX || kind == G_CZ) {
    const uint64_t ma = 1ull << sa;
    const int wb = (int)(b >> 6);
    const uint64_t mb = 1ull << (b & 63);
    uint64_t *xb_p = X + wb * R2 + i;
    uint64_t *zb_p = Z + wb * R2 + i;
    const uint32_t x1 = (*xa_p & ma) != 0, z1 = (*za_p & ma) != 0;
    const uint32_t x2 = (*xb_p & mb) != 0, z2 = (*zb_p & mb) != 0;
    if (kind == G_CX) {
      flip = x1 & z2 & (x2 ^ z1 ^ 1u);
      if (x1) *xb_p ^= mb;
      if (z2) *za_p ^= ma;
    } else {
      flip = x1 & x2 & (z1 ^ z2);
      if (x2) *za_p ^= ma;
      if (x1) *zb_p ^= mb;
    }
  } else {
    const C1Map g = c1_decode(b);
    const uint64_t xw = *xa_p, zw = *za_p;
    const uint32_t xa = (uint32_t)(xw >> sa) & 1u, za = (uint32_t)(zw >> sa) & 1u;
    flip = (g.al & xa) ^ (g.be & za) ^ (g.ga & xa & za);
    const uint32_t nx = (g.m00 & xa) ^ (g.m01 & za), nz = (g.m10 & xa) ^ (g.m11 & za);
    *xa_p = xw ^ ((uint64_t)(xa ^ nx) << sa);
    *za_p = zw ^ ((uint64_t)(za ^ nz) << sa);
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

// One variant with the tableau in LDS; D is the descriptor's access type
// (a kernel argument, or an entry of a device-memory descriptor array read
// through a global-address-space reference).
// Stabilizer row of |+i> = S H|0> after the fragment: img(Y) = i img(X) img(Z)
// for rows in the Hermitian form (-1)^s i^(x.z) X^x Z^z; returns its sign.
template <int W>
__device__ inline uint32_t y_image_sign(const uint64_t *rx, const uint64_t *rz) {
  uint32_t nx = 2u * ((uint32_t)rx[2 * W] & 1u), nz = 2u * ((uint32_t)rz[2 * W] & 1u), cross = 0, pc = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    nx += __popcll(rx[w] & rx[W + w]);
    nz += __popcll(rz[w] & rz[W + w]);
    cross += __popcll(rx[W + w] & rz[w]);
    pc += __popcll((rx[w] ^ rz[w]) & (rx[W + w] ^ rz[W + w]));
  }
  const uint32_t n = 1u + nx + nz + 2u * cross;
  return ((n - pc) & 3u) >> 1;
}

template <int W, int BLOCK, class D>
__device__ void tableau_lds_body(const D &F, uint64_t v, uint64_t *__restrict__ out, uint64_t *smem,
                                 const uint64_t *__restrict__ base = nullptr) {
  const int m = (int)F.m;
  const int R2 = 2 * m;
  const int tid = threadIdx.x;
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
    if (base) {  // the fragment's evolved tableau, shared by its variants
      const uint64_t *row = base + (size_t)i * (2 * W + 1);
#pragma unroll
      for (int w = 0; w < W; ++w) {
        X[w * R2 + i] = row[w];
        Z[w * R2 + i] = row[W + w];
      }
    } else {
#pragma unroll
      for (int w = 0; w < W; ++w) {
        X[w * R2 + i] = (i < m && (i >> 6) == w) ? (1ull << (i & 63)) : 0ull;
        Z[w * R2 + i] = (i >= m && ((i - m) >> 6) == w) ? (1ull << ((i - m) & 63)) : 0ull;
      }
    }
  }
  for (int i = tid; i < m; i += BLOCK) {
    FORM[i] = 0;
    CST[i] = base ? (uint32_t)base[(size_t)(m + i) * (2 * W + 1) + 2 * W] & 1u : 0u;
  }
  if (tid < 64) GROW[tid] = 0;
  if (tid == 0) *X0 = 0;
  __syncthreads();

  // ---- gate phase: every thread updates only its own rows, so no barrier
  // is needed between gates.  Preparations on quantum inputs:
  // |0>, |1> = X|0>, |+> = H|0>, |+i> = S H|0>.  From a shared base tableau
  // they become row substitutions (conjugation is a homomorphism, so the
  // rows equal those of replaying the preparation and the gates):
  // |1>: stabilizer sign flips; |+>: stabilizer <- img(X), destabilizer <-
  // img(Z); |+i>: stabilizer <- i img(X) img(Z), destabilizer <- img(Z).
  if (base) {
    uint64_t t = v;
    for (uint32_t j = 0; j < F.n_axes; ++j) {
      const uint32_t d = (uint32_t)(t % F.axis_radix[j]);
      t /= F.axis_radix[j];
      if (F.axis_side[j] != 1 || d == 0) continue;
      const uint32_t q = F.axis_local[j];
      const uint64_t *rx = base + (size_t)q * (2 * W + 1), *rz = base + (size_t)(m + q) * (2 * W + 1);
      if (d == 1) {
        if (tid == 0) CST[q] ^= 1u;
        continue;
      }
      if (tid < W) {
        const int w = tid;
        X[w * R2 + q] = rz[w];
        Z[w * R2 + q] = rz[W + w];
        X[w * R2 + m + q] = d == 2 ? rx[w] : rx[w] ^ rz[w];
        Z[w * R2 + m + q] = d == 2 ? rx[W + w] : rx[W + w] ^ rz[W + w];
      }
      if (tid == 0) CST[q] = d == 2 ? (uint32_t)rx[2 * W] & 1u : y_image_sign<W>(rx, rz);
    }
  } else {
    uint64_t t = v;
    for (uint32_t j = 0; j < F.n_axes; ++j) {
      const uint32_t d = (uint32_t)(t % F.axis_radix[j]);
      t /= F.axis_radix[j];
      if (F.axis_side[j] != 1 || d == 0) continue;
      const uint32_t q = F.axis_local[j];
      const uint32_t g = prep_c1(d);
      for (int i = tid; i < R2; i += BLOCK) gate_row<W>(X, Z, CST, R2, m, i, G_C1, q, g);
    }
    for (uint32_t g16 = 0; g16 < (F.n_ops + 15) / 16; ++g16) {
      const Ops16 o = load_ops16(F.ops, g16);
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        const uint32_t kind = op_kind(o.w[t]), a = op_q0(o.w[t]), b = op_q1(o.w[t]);
        for (int i = tid; i < R2; i += BLOCK) gate_row<W>(X, Z, CST, R2, m, i, kind, a, b);
      }
    }
  }
  __syncthreads();
  // basis rotations on quantum outputs: X -> H, Y -> S^dag then H, Z -> none
  {
    uint64_t t = v;
    for (uint32_t j = 0; j < F.n_axes; ++j) {
      const uint32_t d = (uint32_t)(t % F.axis_radix[j]);
      t /= F.axis_radix[j];
      if (F.axis_side[j] != 0 || d == 2) continue;
      const uint32_t q = F.axis_local[j];
      const uint32_t g = basis_c1(d);
      for (int i = tid; i < R2; i += BLOCK) gate_row<W>(X, Z, CST, R2, m, i, G_C1, q, g);
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
__global__ __launch_bounds__(BLOCK) void tableau_kernel(const FragDev F, uint64_t v0, uint64_t *__restrict__ models,
                                                        const uint64_t *__restrict__ base) {
  extern __shared__ uint64_t smem[];
  tableau_lds_body<W, BLOCK>(F, v0 + blockIdx.x, models + (size_t)blockIdx.x * model_words(F.n_meas), smem, base);
}

// ---------------------------------------------------------------------------
// Fragments of at most 64 qubits: one wavefront per variant with the whole
// tableau in VGPRs (lane l holds rows l and l + 64).  Gates are pure ALU
// work on the rows' words, the pivot search is a ballot, the pivot row is
// broadcast with readlane, and the deterministic-outcome product is a
// butterfly reduction across the wave: no LDS and no barriers.

__device__ inline uint64_t readlane64(uint64_t v, int lane) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
  return ((uint64_t)hi << 32) | lo;
}

template <int RPL>
__device__ inline void gate_reg(uint64_t (&x)[RPL], uint64_t (&z)[RPL], uint32_t (&cst)[RPL], uint32_t kind,
                                uint32_t a, uint32_t b) {
  if (kind == G_CX || kind == G_CZ) {
    const uint64_t ma = 1ull << a, mb = 1ull << b;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const uint64_t xr = x[r], zr = z[r];
      const uint32_t xa = (uint32_t)(xr >> a) & 1u, za = (uint32_t)(zr >> a) & 1u;
      const uint32_t xb = (uint32_t)(xr >> b) & 1u, zb = (uint32_t)(zr >> b) & 1u;
      if (kind == G_CX) {
        cst[r] ^= xa & zb & (xb ^ za ^ 1u);
        x[r] = xr ^ (xa ? mb : 0ull);
        z[r] = zr ^ (zb ? ma : 0ull);
      } else {
        cst[r] ^= xa & xb & (za ^ zb);
        z[r] = zr ^ (xb ? ma : 0ull) ^ (xa ? mb : 0ull);
      }
    }
    return;
  }
  // fused one-qubit Clifford (every other word, no-ops included)
  const C1Map g = c1_decode(b);
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    const uint32_t xa = (uint32_t)(x[r] >> a) & 1u, za = (uint32_t)(z[r] >> a) & 1u;
    cst[r] ^= (g.al & xa) ^ (g.be & za) ^ (g.ga & xa & za);
    const uint32_t nx = (g.m00 & xa) ^ (g.m01 & za), nz = (g.m10 & xa) ^ (g.m11 & za);
    x[r] ^= (uint64_t)(xa ^ nx) << a;
    z[r] ^= (uint64_t)(za ^ nz) << a;
  }
}

struct Acc1 {
  uint64_t x, z, form;
  uint32_t num;
};

__device__ inline void acc1_combine(Acc1 &L, const Acc1 &R) {
  L.num = (L.num + R.num + 2u * (uint32_t)__popcll(L.z & R.x)) & 3u;
  L.x ^= R.x;
  L.z ^= R.z;
  L.form ^= R.form;
}

template <int RPL, class D>
__device__ void tableau_reg_body(const D &F, uint64_t v, uint64_t *__restrict__ out,
                                 const uint64_t *__restrict__ base = nullptr) {
  const int m = (int)F.m;
  const int R2 = 2 * m;
  const int lane = threadIdx.x & 63;
  const uint32_t n_meas = F.n_meas;
  uint64_t x[RPL], z[RPL], form[RPL];
  uint32_t cst[RPL];
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    const int i = lane + 64 * r;
    if (base) {  // the fragment's evolved tableau (one word per row half)
      const uint64_t *row = base + (size_t)(i < R2 ? i : 0) * 3;
      x[r] = i < R2 ? row[0] : 0ull;
      z[r] = i < R2 ? row[1] : 0ull;
      cst[r] = i < R2 ? (uint32_t)row[2] & 1u : 0u;
    } else {
      x[r] = (i < m) ? (1ull << i) : 0ull;
      z[r] = (i >= m && i < R2) ? (1ull << (i - m)) : 0ull;
      cst[r] = 0;
    }
    form[r] = 0;
  }
  if (base) {  // preparations as row substitutions (see the LDS body)
    uint64_t t = v;
    for (uint32_t j = 0; j < F.n_axes; ++j) {
      const uint32_t d = (uint32_t)(t % F.axis_radix[j]);
      t /= F.axis_radix[j];
      if (F.axis_side[j] != 1 || d == 0) continue;
      const int q = (int)F.axis_local[j];
      const uint64_t *rx = base + (size_t)q * 3, *rz = base + (size_t)(m + q) * 3;
#pragma unroll
      for (int r = 0; r < RPL; ++r) {
        const int i = lane + 64 * r;
        if (i == m + q) {
          if (d == 1) {
            cst[r] ^= 1u;
          } else {
            x[r] = d == 2 ? rx[0] : rx[0] ^ rz[0];
            z[r] = d == 2 ? rx[1] : rx[1] ^ rz[1];
            cst[r] = d == 2 ? (uint32_t)rx[2] & 1u : y_image_sign<1>(rx, rz);
          }
        } else if (i == q && d >= 2) {
          x[r] = rz[0];
          z[r] = rz[1];
          cst[r] = (uint32_t)rz[2] & 1u;
        }
      }
    }
  } else {  // preparations: |1> = X|0>, |+> = H|0>, |+i> = S H|0>
    uint64_t t = v;
    for (uint32_t j = 0; j < F.n_axes; ++j) {
      const uint32_t d = (uint32_t)(t % F.axis_radix[j]);
      t /= F.axis_radix[j];
      if (F.axis_side[j] != 1 || d == 0) continue;
      gate_reg<RPL>(x, z, cst, G_C1, F.axis_local[j], prep_c1(d));
    }
  }
  if (!base) {
    const uint32_t n16 = (F.n_ops + 15) / 16;
    for (uint32_t g16 = 0; g16 < n16; ++g16) {
      const Ops16 o = load_ops16(F.ops, g16);
#pragma unroll
      for (int t = 0; t < 16; ++t) gate_reg<RPL>(x, z, cst, op_kind(o.w[t]), op_q0(o.w[t]), op_q1(o.w[t]));
    }
  }
  {  // basis rotations: X -> H, Y -> S^dag then H
    uint64_t t = v;
    for (uint32_t j = 0; j < F.n_axes; ++j) {
      const uint32_t d = (uint32_t)(t % F.axis_radix[j]);
      t /= F.axis_radix[j];
      if (F.axis_side[j] != 0 || d == 2) continue;
      gate_reg<RPL>(x, z, cst, G_C1, F.axis_local[j], basis_c1(d));
    }
  }
  uint64_t x0 = 0, randmask = 0, my_grow = 0;
  for (uint32_t j = 0; j < n_meas; ++j) {
    const uint32_t a = F.meas[j];
    const uint64_t ma = 1ull << a;
    uint64_t bal[RPL];
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int i = lane + 64 * r;
      bal[r] = __ballot(i >= m && i < R2 && (x[r] & ma));
    }
    int p = -1;
#pragma unroll
    for (int r = RPL - 1; r >= 0; --r)
      if (bal[r]) p = 64 * r + __ffsll((unsigned long long)bal[r]) - 1;
    if (p >= 0) {
      // random: row p multiplies into every other row with x_a = 1
      const int pl = p & 63, pr = p >> 6;
      uint64_t xsel = x[0], zsel = z[0], fsel = form[0];
      uint32_t csel = cst[0];
      if (RPL > 1 && pr == 1) {
        xsel = x[RPL - 1];
        zsel = z[RPL - 1];
        fsel = form[RPL - 1];
        csel = cst[RPL - 1];
      }
      const uint64_t xp = readlane64(xsel, pl), zp = readlane64(zsel, pl), formp = readlane64(fsel, pl);
      const uint32_t cstp = (uint32_t)__builtin_amdgcn_readlane((int)csel, pl);
      const uint32_t pcp = (uint32_t)__popcll(xp & zp);
#pragma unroll
      for (int r = 0; r < RPL; ++r) {
        const int i = lane + 64 * r;
        if (i < R2 && i != p && (x[r] & ma)) {
          const uint64_t xi = x[r], zi = z[r];
          const uint64_t xn = xi ^ xp, zn = zi ^ zp;
          const uint32_t num = 2u * cstp + pcp + 2u * cst[r] + (uint32_t)__popcll(xi & zi) +
                               2u * (uint32_t)__popcll(zp & xi) - (uint32_t)__popcll(xn & zn);
          cst[r] = (num & 3u) >> 1;
          form[r] ^= formp;
          x[r] = xn;
          z[r] = zn;
        }
      }
      const int q = p - m;  // destabilizer row paired with the pivot (q < 64: row set 0)
      if (lane == q) {
        x[0] = xp;
        z[0] = zp;
      }
#pragma unroll
      for (int r = 0; r < RPL; ++r)
        if (lane == pl && r == pr) {
          x[r] = 0;
          z[r] = ma;
          form[r] = 1ull << j;
          cst[r] = 0;
        }
      randmask |= 1ull << j;
      if (lane == (int)j) my_grow = 1ull << j;
    } else {
      // deterministic: product of the stabilizers paired with destabilizers
      // that have x_a = 1 (destabilizers are rows 0..m-1 < 64: row set 0)
      const uint64_t dsel = __ballot(lane < m && (x[0] & ma));
      Acc1 acc{0, 0, 0, 0};
#pragma unroll
      for (int r = 0; r < RPL; ++r) {
        const int i = lane + 64 * r;
        if (i >= m && i < R2 && ((dsel >> (i - m)) & 1ull)) {
          Acc1 row{x[r], z[r], form[r], (2u * cst[r] + (uint32_t)__popcll(x[r] & z[r])) & 3u};
          acc1_combine(acc, row);
        }
      }
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        Acc1 o;
        o.x = __shfl_xor(acc.x, off);
        o.z = __shfl_xor(acc.z, off);
        o.form = __shfl_xor(acc.form, off);
        o.num = (uint32_t)__shfl_xor((int)acc.num, off);
        if ((lane & off) == 0) {
          acc1_combine(acc, o);
        } else {
          acc1_combine(o, acc);
          acc = o;
        }
      }
      x0 |= (uint64_t)((acc.num & 3u) >> 1) << j;
      if (lane == (int)j) my_grow = acc.form;
    }
  }
  if (lane == 0) {
    out[0] = x0;
    out[1] = randmask;
  }
  uint64_t col = 0;
  for (uint32_t j = 0; j < n_meas; ++j) col |= ((readlane64(my_grow, (int)j) >> lane) & 1ull) << j;
  if ((uint32_t)lane < n_meas) out[2 + lane] = col;
}

template <int RPL>
__global__ __launch_bounds__(64) void tableau_reg_kernel(const FragDev F, uint64_t v0, uint64_t *__restrict__ models,
                                                         const uint64_t *__restrict__ base) {
  tableau_reg_body<RPL>(F, v0 + blockIdx.x, models + (size_t)blockIdx.x * model_words(F.n_meas), base);
}

// ---------------------------------------------------------------------------
// Batched evaluation: one persistent launch over the Clifford variants of
// many circuits.  Workgroups pull (descriptor, variant) items from an atomic
// queue (items are pre-sorted by cost, longest first) until it runs dry;
// every wave sees the same item index, so the exit is uniform.
typedef __attribute__((address_space(1))) const FragDev g_FragDev;

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void tableau_batch_kernel(const FragDev *__restrict__ descs,
                                                              const BatchItem *__restrict__ items,
                                                              uint32_t n_items, uint32_t *__restrict__ counter,
                                                              uint64_t *__restrict__ models, uint32_t use_reg,
                                                              const uint64_t *__restrict__ bases) {
  extern __shared__ uint64_t smem[];
  __shared__ uint32_t s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1u);
    __syncthreads();
    const uint32_t it = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_item);
    __syncthreads();
    if (it >= n_items) break;
    const __attribute__((address_space(1))) const BatchItem &item = ((const __attribute__((address_space(1))) const BatchItem *)items)[it];
    const uint32_t di = item.desc;
    const uint64_t v = item.variant;
    uint64_t *out = models + item.model_off;
    const uint64_t *base = bases ? bases + item.base_off : nullptr;
    const g_FragDev &F = ((const g_FragDev *)descs)[di];
    const uint32_t m = F.m;
    if (BLOCK == 64 && use_reg && 2 * m <= 64) {
      tableau_reg_body<1>(F, v, out, base);
    } else if (BLOCK == 64 && use_reg && m <= 64) {
      tableau_reg_body<2>(F, v, out, base);
    } else {
      const uint32_t W = (m + 63) / 64;
      if (W <= 1)
        tableau_lds_body<1, BLOCK>(F, v, out, smem, base);
      else if (W <= 2)
        tableau_lds_body<2, BLOCK>(F, v, out, smem, base);
      else if (W <= 4)
        tableau_lds_body<4, BLOCK>(F, v, out, smem, base);
      else
        tableau_lds_body<8, BLOCK>(F, v, out, smem, base);
    }
    __syncthreads();
  }
}

__global__ void fill_u32_kernel(uint32_t *p, uint64_t n, uint32_t value) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

template <int RPL>
hipError_t launch_reg(const FragDev &h, uint64_t v0, uint64_t nv, uint64_t *models, const uint64_t *base,
                      hipStream_t s) {
  for (uint64_t done = 0; done < nv;) {
    uint64_t chunk = nv - done;
    if (chunk > (1ull << 30)) chunk = 1ull << 30;
    hipLaunchKernelGGL((tableau_reg_kernel<RPL>), dim3((unsigned)chunk), dim3(64), 0, s, h, v0 + done,
                       models + done * model_words(h.n_meas), base);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    done += chunk;
  }
  return hipSuccess;
}

template <int W, int BLOCK>
hipError_t launch_w(const FragDev &h, uint64_t v0, uint64_t nv, uint64_t *models, const uint64_t *base,
                    hipStream_t s) {
  const size_t lds = tableau_lds<W, BLOCK>(h.m);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute((const void *)tableau_kernel<W, BLOCK>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  for (uint64_t done = 0; done < nv;) {
    uint64_t chunk = nv - done;
    if (chunk > (1ull << 30)) chunk = 1ull << 30;
    hipLaunchKernelGGL((tableau_kernel<W, BLOCK>), dim3((unsigned)chunk), dim3(BLOCK), lds, s, h,
                       v0 + done, models + done * model_words(h.n_meas), base);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    done += chunk;
  }
  return hipSuccess;
}

}  // namespace

hipError_t launch_tableau(const FragDev &h, uint64_t v0, uint64_t nv, uint64_t *models, hipStream_t s,
                          const uint64_t *base) {
  if (h.n_meas > (uint32_t)kMaxMeas) return hipErrorInvalidValue;
  const uint32_t W = (h.m + 63) / 64;
  if (2 * h.m <= 64) return launch_reg<1>(h, v0, nv, models, base, s);
  if (h.m <= 64) return launch_reg<2>(h, v0, nv, models, base, s);
  if (W <= 2) return launch_w<2, 128>(h, v0, nv, models, base, s);
  if (W <= 4) return launch_w<4, 256>(h, v0, nv, models, base, s);
  if (W <= 8) return launch_w<8, 256>(h, v0, nv, models, base, s);
  return hipErrorInvalidValue;
}

size_t tableau_batch_lds(uint32_t max_m, uint32_t block) {
  const uint32_t W = (max_m + 63) / 64;
  auto pick = [&](auto wtag) -> size_t {
    constexpr int Wc = decltype(wtag)::value;
    if (block == 64) return tableau_lds<Wc, 64>(max_m);
    if (block == 128) return tableau_lds<Wc, 128>(max_m);
    return tableau_lds<Wc, 256>(max_m);
  };
  if (W <= 1) return pick(std::integral_constant<int, 1>());
  if (W <= 2) return pick(std::integral_constant<int, 2>());
  if (W <= 4) return pick(std::integral_constant<int, 4>());
  return pick(std::integral_constant<int, 8>());
}

hipError_t launch_tableau_batch(const FragDev *descs, const BatchItem *items, uint32_t n_items, uint32_t *counter,
                                uint64_t *models, uint32_t max_m, uint32_t block, uint32_t grid, uint32_t use_reg,
                                const uint64_t *bases, hipStream_t s) {
  if (max_m > 512 || grid == 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(64), 0, s, counter, (uint64_t)1, 0u);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t lds = tableau_batch_lds(max_m, block);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  switch (block) {
    case 64:
      (void)hipFuncSetAttribute((const void *)tableau_batch_kernel<64>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds);
      hipLaunchKernelGGL(tableau_batch_kernel<64>, dim3(grid), dim3(64), lds, s, descs, items, n_items, counter,
                         models, use_reg, bases);
      break;
    case 128:
      (void)hipFuncSetAttribute((const void *)tableau_batch_kernel<128>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds);
      hipLaunchKernelGGL(tableau_batch_kernel<128>, dim3(grid), dim3(128), lds, s, descs, items, n_items, counter,
                         models, 0u, bases);
      break;
    case 256:
      (void)hipFuncSetAttribute((const void *)tableau_batch_kernel<256>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds);
      hipLaunchKernelGGL(tableau_batch_kernel<256>, dim3(grid), dim3(256), lds, s, descs, items, n_items, counter,
                         models, 0u, bases);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t value, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<uint64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(fill_u32_kernel, dim3(blocks), dim3(256), 0, s, p, n, value);
  return hipGetLastError();
}

}  // namespace ccut

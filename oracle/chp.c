/*
 * Literal Aaronson-Gottesman stabilizer tableau ("CHP"), S. Aaronson and
 * D. Gottesman, "Improved simulation of stabilizer circuits", PRA 70,
 * 052328 (2004) -- the Clifford simulator the paper builds on (Sec. III-B).
 *
 * Test infrastructure for the CPU oracle: plain, slow, one byte per bit.
 * Rows 0..n-1 are destabilizers (initially X_i), rows n..2n-1 stabilizers
 * (initially Z_i), row 2n is the scratch row; r[] holds the sign bits.
 * Only the paper's three primitive updates (CNOT, Hadamard, phase) touch the
 * tableau; every other Clifford gate is composed from them:
 *   Z = S S,  X = H Z H,  Y ~ X Z (same conjugation),  S^dag = S S S,
 *   CZ(a, b) = H(b) CNOT(a, b) H(b).
 * Measurement follows the AG procedure: a random outcome (some stabilizer
 * anticommutes with Z_a) takes the caller-supplied bit; a deterministic one
 * is read from the scratch row after the rowsum chain.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int n;
  uint8_t *x; /* (2n+1) x n */
  uint8_t *z; /* (2n+1) x n */
  uint8_t *r; /* 2n+1 */
} chp_tab;

#define XB(t, i, j) ((t)->x[(size_t)(i) * (size_t)(t)->n + (size_t)(j)])
#define ZB(t, i, j) ((t)->z[(size_t)(i) * (size_t)(t)->n + (size_t)(j)])

chp_tab *chp_new(int n) {
  chp_tab *t = (chp_tab *)calloc(1, sizeof(chp_tab));
  size_t rows = (size_t)(2 * n + 1);
  t->n = n;
  t->x = (uint8_t *)calloc(rows * (size_t)n + 1, 1);
  t->z = (uint8_t *)calloc(rows * (size_t)n + 1, 1);
  t->r = (uint8_t *)calloc(rows, 1);
  for (int i = 0; i < n; i++) {
    XB(t, i, i) = 1;
    ZB(t, n + i, i) = 1;
  }
  return t;
}

void chp_free(chp_tab *t) {
  if (!t) return;
  free(t->x);
  free(t->z);
  free(t->r);
  free(t);
}

void chp_copy_into(chp_tab *dst, const chp_tab *src) {
  size_t rows = (size_t)(2 * src->n + 1);
  memcpy(dst->x, src->x, rows * (size_t)src->n);
  memcpy(dst->z, src->z, rows * (size_t)src->n);
  memcpy(dst->r, src->r, rows);
}

chp_tab *chp_clone(const chp_tab *src) {
  chp_tab *t = chp_new(src->n);
  chp_copy_into(t, src);
  return t;
}

/* ---- the three primitive updates, applied to rows 0..2n-1 ---- */
static void prim_cnot(chp_tab *t, int a, int b) {
  for (int i = 0; i < 2 * t->n; i++) {
    t->r[i] ^= XB(t, i, a) & ZB(t, i, b) & (XB(t, i, b) ^ ZB(t, i, a) ^ 1);
    XB(t, i, b) ^= XB(t, i, a);
    ZB(t, i, a) ^= ZB(t, i, b);
  }
}

static void prim_h(chp_tab *t, int a) {
  for (int i = 0; i < 2 * t->n; i++) {
    uint8_t xa = XB(t, i, a), za = ZB(t, i, a);
    t->r[i] ^= xa & za;
    XB(t, i, a) = za;
    ZB(t, i, a) = xa;
  }
}

static void prim_s(chp_tab *t, int a) {
  for (int i = 0; i < 2 * t->n; i++) {
    t->r[i] ^= XB(t, i, a) & ZB(t, i, a);
    ZB(t, i, a) ^= XB(t, i, a);
  }
}

/* gate kinds: 0 H, 1 S, 2 SDG, 3 X, 4 Y, 5 Z, 6 CX, 7 CZ */
int chp_gate(chp_tab *t, int kind, int a, int b) {
  switch (kind) {
  case 0: prim_h(t, a); break;
  case 1: prim_s(t, a); break;
  case 2: prim_s(t, a); prim_s(t, a); prim_s(t, a); break;
  case 3: prim_h(t, a); prim_s(t, a); prim_s(t, a); prim_h(t, a); break;
  case 4: /* Y = i X Z: conjugation by X after Z */
    prim_s(t, a); prim_s(t, a);
    prim_h(t, a); prim_s(t, a); prim_s(t, a); prim_h(t, a);
    break;
  case 5: prim_s(t, a); prim_s(t, a); break;
  case 6: prim_cnot(t, a, b); break;
  case 7: prim_h(t, b); prim_cnot(t, a, b); prim_h(t, b); break;
  default: return -1;
  }
  return 0;
}

/* phase exponent of the product of single-qubit Paulis (x1,z1)(x2,z2) */
static int g_fn(int x1, int z1, int x2, int z2) {
  if (x1 == 0 && z1 == 0) return 0;
  if (x1 == 1 && z1 == 1) return z2 - x2;
  if (x1 == 1 && z1 == 0) return z2 * (2 * x2 - 1);
  return x2 * (1 - 2 * z2);
}

/* row h <- row i * row h, with the AG sign rule */
static void rowsum(chp_tab *t, int h, int i) {
  int sum = 2 * t->r[h] + 2 * t->r[i];
  for (int j = 0; j < t->n; j++)
    sum += g_fn(XB(t, i, j), ZB(t, i, j), XB(t, h, j), ZB(t, h, j));
  sum %= 4;
  if (sum < 0) sum += 4;
  t->r[h] = (uint8_t)(sum >= 2 ? 1 : 0);
  for (int j = 0; j < t->n; j++) {
    XB(t, h, j) ^= XB(t, i, j);
    ZB(t, h, j) ^= ZB(t, i, j);
  }
}

int chp_is_random(const chp_tab *t, int a) {
  for (int p = t->n; p < 2 * t->n; p++)
    if (XB(t, p, a)) return 1;
  return 0;
}

/* Measure qubit a in Z.  A random outcome equals `bit`. */
int chp_measure(chp_tab *t, int a, int bit, int *was_random) {
  int n = t->n, p = -1;
  for (int q = n; q < 2 * n; q++)
    if (XB(t, q, a)) { p = q; break; }
  if (p >= 0) {
    for (int i = 0; i < 2 * n; i++)
      if (i != p && XB(t, i, a)) rowsum(t, i, p);
    memcpy(&XB(t, p - n, 0), &XB(t, p, 0), (size_t)n);
    memcpy(&ZB(t, p - n, 0), &ZB(t, p, 0), (size_t)n);
    t->r[p - n] = t->r[p];
    memset(&XB(t, p, 0), 0, (size_t)n);
    memset(&ZB(t, p, 0), 0, (size_t)n);
    ZB(t, p, a) = 1;
    t->r[p] = (uint8_t)(bit & 1);
    if (was_random) *was_random = 1;
    return bit & 1;
  }
  memset(&XB(t, 2 * n, 0), 0, (size_t)n);
  memset(&ZB(t, 2 * n, 0), 0, (size_t)n);
  t->r[2 * n] = 0;
  for (int i = 0; i < n; i++)
    if (XB(t, i, a)) rowsum(t, 2 * n, i + n);
  if (was_random) *was_random = 0;
  return t->r[2 * n];
}

void chp_dump(const chp_tab *t, uint8_t *x, uint8_t *z, uint8_t *r) {
  size_t rows = (size_t)(2 * t->n + 1);
  memcpy(x, t->x, rows * (size_t)t->n);
  memcpy(z, t->z, rows * (size_t)t->n);
  memcpy(r, t->r, rows);
}

/* ---- Philox4x32-10, from the SC'11 definition ---- */
static void philox(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int rnd = 0; rnd < 10; rnd++) {
    if (rnd) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

void chp_philox(const uint32_t *ctr, const uint32_t *key, uint32_t *out) { philox(ctr, key, out); }

static int shot_bit(uint64_t seed, uint64_t vid, uint64_t shot, int a) {
  uint32_t ctr[4] = {(uint32_t)(a >> 5), (uint32_t)(shot >> 2), (uint32_t)vid, (uint32_t)(vid >> 32)};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t o[4];
  philox(ctr, key, o);
  return (int)((o[shot & 3] >> (a & 31)) & 1u);
}

/*
 * Per-shot literal sampling: for every shot, start again from the given
 * (already prepared and rotated) tableau and measure meas[0..nm-1] in order.
 * out[(s - shot0) * nm + j] = outcome of measurement j of shot s.
 */
void chp_sample(const chp_tab *t0, const int *meas, int nm, uint64_t seed, uint64_t vid,
                uint64_t shot0, uint64_t nshots, uint8_t *out) {
  chp_tab *t = chp_clone(t0);
  for (uint64_t s = shot0; s < shot0 + nshots; s++) {
    chp_copy_into(t, t0);
    for (int j = 0; j < nm; j++) {
      int bit = chp_is_random(t, meas[j]) ? shot_bit(seed, vid, s, j) : 0;
      out[(s - shot0) * (uint64_t)nm + (uint64_t)j] = (uint8_t)chp_measure(t, meas[j], bit, NULL);
    }
  }
  chp_free(t);
}

/* Same, but accumulate a histogram over the nm-bit outcome index
 * (bit j of the index = measurement j).  hist has 2^nm entries. */
void chp_sample_hist(const chp_tab *t0, const int *meas, int nm, uint64_t seed, uint64_t vid,
                     uint64_t nshots, uint64_t *hist) {
  chp_tab *t = chp_clone(t0);
  for (uint64_t s = 0; s < nshots; s++) {
    chp_copy_into(t, t0);
    uint64_t idx = 0;
    for (int j = 0; j < nm; j++) {
      int bit = chp_is_random(t, meas[j]) ? shot_bit(seed, vid, s, j) : 0;
      idx |= (uint64_t)chp_measure(t, meas[j], bit, NULL) << j;
    }
    hist[idx] += 1;
  }
  chp_free(t);
}

/* Exact outcome distribution by branching on both values of every random
 * measurement (2^R leaves, each of probability 2^-R).  table has 2^nm
 * entries and is accumulated into. */
static void branch(const chp_tab *t, const int *meas, int nm, int j, uint64_t idx, double prob,
                   double *table) {
  if (j == nm) { table[idx] += prob; return; }
  if (!chp_is_random(t, meas[j])) {
    chp_tab *c = chp_clone(t);
    int o = chp_measure(c, meas[j], 0, NULL);
    branch(c, meas, nm, j + 1, idx | ((uint64_t)o << j), prob, table);
    chp_free(c);
    return;
  }
  for (int bit = 0; bit < 2; bit++) {
    chp_tab *c = chp_clone(t);
    int o = chp_measure(c, meas[j], bit, NULL);
    branch(c, meas, nm, j + 1, idx | ((uint64_t)o << j), prob * 0.5, table);
    chp_free(c);
  }
}

void chp_exact(const chp_tab *t0, const int *meas, int nm, double *table) {
  branch(t0, meas, nm, 0, 0, 1.0, table);
}

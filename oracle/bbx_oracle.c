/*
 * bbx_oracle.c -- plain, slow, single-threaded CPU oracle of the bit-box
 * particle compressor (arXiv 2404.02826), FP64 arithmetic throughout.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg; never by the product path.  It shares no code
 * with the HIP library.  Build: -O2 -ffp-contract=off, no fast-math.
 *
 * Each step follows the paper's method in its order, with the readings chosen
 * where the paper is silent:
 *   1. range and bound      Sec. 3 (absolute / value-range relative bound)
 *   2. quantize             Sec. 3 (linear-scale quantization, bins of 2*eb)
 *   3. k-d median partition Sec. 4.1 (median split, median on the larger side,
 *                           stop at <= r particles), round-robin split axis,
 *                           ties by original particle index
 *   4. bit box per leaf     Sec. 4.1 (AABB, reference = particle nearest the
 *                           AABB centre, Eq. 2 bit widths)
 *   5. offsets + packing    Sec. 4.2 (sequence layout, 5/6-bit width fields;
 *                           storage-cost model) in a structure-of-arrays form;
 *                           the reference stored as its codes, or (ref_mode
 *                           1) losslessly as its original coordinates
 *   6. unpack + dequantize  Sec. 3 (reconstruction at the bin centre)
 *
 * Parity pins live in tests/: a worked example of Sec. 4.1, a pure-Python
 * brute-force re-derivation on tiny inputs, closed forms (Eq. 1-3), the error
 * bound, and mutation tests that build this file with -DBBXO_MUTANT=k to
 * plant one plausible mistake k and check that some pin catches it.
 *
 * Parity unpinned (readings, checked only against the brute-force
 * restatement): the direction of the sequence reordering in
 * bbxo_export_sequences_reordered (ascending sum of widths) and the value of
 * the 32-bit end mark of the exported sequence layout (all ones).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "bbx_oracle.h"

#ifndef BBXO_MUTANT
#define BBXO_MUTANT 0 /* 0: faithful; k > 0: plant mistake k (mutation tests only) */
#endif
#define MUT(k) (BBXO_MUTANT == (k))

#define MAGIC 0x31584242u /* bytes 'B','B','X','1' */
#define HEADER_BYTES 128u

/* ------------------------------------------------------------------ helpers */

static uint32_t bitlen64(uint64_t v) {
  uint32_t b = 0;
  while (v) {
    b++;
    v >>= 1;
  }
  return b;
}

/* Eq. 2: m = ceil(log2(D + 1/2) + 1), D = largest |offset| from the reference
 * in bins of width 2*eb.  For 2^(k-1) <= D < 2^k, D + 1/2 lies strictly between
 * 2^(k-1) and 2^k, so the ceiling is k + 1 = bitlen(D) + 1.  For D = 0 the
 * expression is exactly 0. */
uint32_t bbxo_bits_for_offset(uint64_t D) {
  if (D == 0) return 0;
#if MUT(6)
  return bitlen64(D);
#else
  return bitlen64(D) + 1;
#endif
}

static void put_u16le(uint8_t* b, uint32_t v) { b[0] = (uint8_t)v; b[1] = (uint8_t)(v >> 8); }
static void put_u32le(uint8_t* b, uint32_t v) {
  for (int k = 0; k < 4; k++) b[k] = (uint8_t)(v >> (8 * k));
}
static void put_u64le(uint8_t* b, uint64_t v) {
  for (int k = 0; k < 8; k++) b[k] = (uint8_t)(v >> (8 * k));
}
static void put_f64le(uint8_t* b, double v) {
  uint64_t u;
  memcpy(&u, &v, 8);
  put_u64le(b, u);
}
static uint32_t get_u16le(const uint8_t* b) { return (uint32_t)b[0] | ((uint32_t)b[1] << 8); }
static uint32_t get_u32le(const uint8_t* b) {
  uint32_t v = 0;
  for (int k = 0; k < 4; k++) v |= (uint32_t)b[k] << (8 * k);
  return v;
}
static uint64_t get_u64le(const uint8_t* b) {
  uint64_t v = 0;
  for (int k = 0; k < 8; k++) v |= (uint64_t)b[k] << (8 * k);
  return v;
}
static double get_f64le(const uint8_t* b) {
  uint64_t u = get_u64le(b);
  double v;
  memcpy(&v, &u, 8);
  return v;
}

/* One bit at a time: bit i of a section is bit (i mod 8) of byte i/8, which is
 * bit (i mod 64) of the little-endian 64-bit word i/64. */
static void put_bits(uint8_t* sec, uint64_t pos, uint64_t v, uint32_t nb) {
  for (uint32_t k = 0; k < nb; k++)
    if ((v >> k) & 1u) sec[(pos + k) >> 3] |= (uint8_t)(1u << ((pos + k) & 7u));
}
static uint64_t get_bits(const uint8_t* sec, uint64_t pos, uint32_t nb) {
  uint64_t v = 0;
  for (uint32_t k = 0; k < nb; k++)
    if ((sec[(pos + k) >> 3] >> ((pos + k) & 7u)) & 1u) v |= (uint64_t)1 << k;
  return v;
}

/* ------------------------------------------------------------------ params */

typedef struct {
  uint64_t n;
  uint32_t dims;
  int dtype, eb_mode;
  uint32_t r, mbits;
  double eb_user, eb_abs, eb_eff, w, inv_w;
  double lo[3], hi[3];
  uint32_t G[3];
} params_t;

static double coord(const void* pos, const params_t* p, int layout, uint64_t i, uint32_t d) {
  uint64_t k = (layout == 0) ? i * p->dims + d : (uint64_t)d * p->n + i;
  return p->dtype == 0 ? (double)((const float*)pos)[k] : ((const double*)pos)[k];
}

/* Bits of one stored coordinate (M of Sec. 4.2), and a coordinate's bits. */
static uint32_t coord_bits(int dtype) { return dtype == 0 ? 32u : 64u; }
static uint64_t coord_raw(const void* pos, const params_t* p, int layout, uint64_t i, uint32_t d) {
  uint64_t k = (layout == 0) ? i * p->dims + d : (uint64_t)d * p->n + i;
  if (p->dtype == 0) {
    uint32_t u;
    memcpy(&u, (const float*)pos + k, 4);
    return u;
  }
  uint64_t u;
  memcpy(&u, (const double*)pos + k, 8);
  return u;
}

/* Sec. 3 quantization: index of the bin of width w (= 2*eb_eff) holding x,
 * bins centred on lo + k*w; round-half-up, three separately rounded FP64
 * operations. */
static double quantize_real(double x, double lo, double inv_w) {
  double t = (x - lo) * inv_w + 0.5;
  return floor(t);
}

/* Steps 1-2: per-axis range, error bound, bin width, code widths G_d. */
static int range_and_bound(const void* pos, int layout, params_t* p) {
  uint32_t dims = p->dims;
  for (uint32_t d = 0; d < 3; d++) p->lo[d] = p->hi[d] = 0.0, p->G[d] = 0;
  p->eb_abs = p->eb_eff = p->w = p->inv_w = 0.0;
  if (p->n == 0) {
    p->eb_abs = (p->eb_mode == 1) ? p->eb_user : 0.0;
    return BBXO_OK;
  }
  for (uint32_t d = 0; d < dims; d++) p->lo[d] = p->hi[d] = coord(pos, p, layout, 0, d);
  for (uint64_t i = 0; i < p->n; i++)
    for (uint32_t d = 0; d < dims; d++) {
      double v = coord(pos, p, layout, i, d);
      if (!isfinite(v)) return BBXO_EINVAL;
      if (v < p->lo[d]) p->lo[d] = v;
      if (v > p->hi[d]) p->hi[d] = v;
    }
  /* -0.0 and +0.0 compare equal; make the stored origin +0.0 either way */
  for (uint32_t d = 0; d < dims; d++) {
    p->lo[d] = p->lo[d] + 0.0;
    p->hi[d] = p->hi[d] + 0.0;
  }
  /* Delta_max: the largest coordinate range over all axes (Sec. 3) */
  double delta = 0.0;
  for (uint32_t d = 0; d < dims; d++) {
    double rg = p->hi[d] - p->lo[d];
#if MUT(15)
    if (d == 0 || rg < delta) delta = rg;
#else
    if (rg > delta) delta = rg;
#endif
  }
  p->eb_abs = (p->eb_mode == 0) ? p->eb_user * delta : p->eb_user;
  if (!isfinite(delta) || !isfinite(p->eb_abs)) return BBXO_EBOUND;
  if (delta == 0.0) return BBXO_OK; /* all particles identical: exact, w = 0 */

  /* Guard: the bound must survive FP64 rounding of quantize/dequantize and the
   * final rounding to the input type.  guard = ulp_T(A)/2 (T = f32 only) +
   * A * 2^-48, A = largest magnitude of any coordinate or reconstruction. */
  double amax = 0.0;
  for (uint32_t d = 0; d < dims; d++) {
    double a = fabs(p->lo[d]) > fabs(p->hi[d]) ? fabs(p->lo[d]) : fabs(p->hi[d]);
    if (a > amax) amax = a;
  }
  amax = amax + p->eb_abs;
  double guard = ldexp(amax, -48);
  if (p->dtype == 0) {
    int e = 0;
    (void)frexp(amax, &e); /* amax = f * 2^e, f in [1/2, 1): f32 ulp is 2^(e-24) */
#if MUT(18)
    double half_ulp = ldexp(1.0, e - 24); /* a whole ulp */
#else
    double half_ulp = ldexp(1.0, e - 25);
#endif
    if (half_ulp < ldexp(1.0, -150)) half_ulp = ldexp(1.0, -150);
    guard = guard + half_ulp;
  }
  p->eb_eff = p->eb_abs - guard;
  if (!(p->eb_eff > 0.0)) return BBXO_EBOUND;
#if MUT(9)
  p->w = p->eb_eff;
#else
  p->w = 2.0 * p->eb_eff;
#endif
  p->inv_w = 1.0 / p->w;
  if (!isfinite(p->w) || !isfinite(p->inv_w) || !(p->inv_w > 0.0)) return BBXO_EBOUND;
  /* the largest code of axis d is the code of hi_d (quantization is monotone) */
  for (uint32_t d = 0; d < dims; d++) {
    double qm = quantize_real(p->hi[d], p->lo[d], p->inv_w);
    if (!(qm < 1073741824.0)) return BBXO_EBOUND; /* codes must stay below 2^30 */
    p->G[d] = bitlen64((uint64_t)qm);
#if MUT(14)
    if (p->G[d] > 0) p->G[d] -= 1;
#endif
  }
  return BBXO_OK;
}

/* ------------------------------------------------------------------ tree */

typedef struct {
  const uint32_t* q; /* [dims][n] */
  uint64_t n;
  uint32_t dims, r;
  uint32_t* order;  /* tree order being built, [n] */
  uint64_t* keys;   /* scratch, [n] */
  uint32_t* tmp;    /* scratch, [n] */
  uint32_t* leaf_start;
  uint32_t* leaf_size;
  uint64_t nleaves, cap;
  int fail;
  int rule;         /* split rule, see kd_split */
  uint64_t nb;      /* rule 2: leaves of the whole tree, ceil(n / r) */
} tree_t;

/* What a node knows besides its members: rule 2 the leaves [i0, i1) it will
 * hold, rule 3 its cell, the codes lo[d] .. lo[d] + 2^lg[d] - 1 per axis. */
typedef struct {
  uint64_t i0, i1;
  uint32_t lo[3], lg[3];
} node_t;

static int cmp_u64(const void* a, const void* b) {
  uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
  return (x > y) - (x < y);
}

/* (q_d, original index) as one ordered 64-bit key: codes < 2^30, index < 2^32 */
static uint64_t split_key(const tree_t* t, uint32_t i, uint32_t d) {
#if MUT(2)
  return ((uint64_t)t->q[(uint64_t)d * t->n + i] << 32) | (uint64_t)(0xffffffffu - i);
#else
  return ((uint64_t)t->q[(uint64_t)d * t->n + i] << 32) | (uint64_t)i;
#endif
}

static void add_leaf(tree_t* t, uint64_t start, uint64_t s) {
  if (t->nleaves >= t->cap) {
    t->fail = 1;
    return;
  }
  t->leaf_start[t->nleaves] = (uint32_t)start;
  t->leaf_size[t->nleaves] = (uint32_t)s;
  t->nleaves++;
}

/* Stable split of S[0, s) along axis d at rank k: the member of rank k in
 * (q_d, index) order and everything after it form the right child; both
 * children keep ascending original index.  Returns the left size (k). */
static uint64_t split_rank(tree_t* t, uint32_t* S, uint64_t s, uint32_t d, uint64_t k) {
  for (uint64_t j = 0; j < s; j++) t->keys[j] = split_key(t, S[j], d);
  qsort(t->keys, (size_t)s, sizeof(uint64_t), cmp_u64);
#if MUT(1)
  uint64_t med = k == s / 2 ? t->keys[(s - 1) / 2] + 1 : t->keys[k]; /* median joins the left */
#else
  uint64_t med = t->keys[k];
#endif
  uint64_t nl = 0;
  for (uint64_t j = 0; j < s; j++)
    if (split_key(t, S[j], d) < med) t->tmp[nl++] = S[j];
  uint64_t m = nl;
  for (uint64_t j = 0; j < s; j++)
    if (!(split_key(t, S[j], d) < med)) t->tmp[m++] = S[j];
  memcpy(S, t->tmp, (size_t)s * sizeof(uint32_t));
  return nl;
}

/* Stable split of S[0, s) by value: codes q_d < mid go left. */
static uint64_t split_value(tree_t* t, uint32_t* S, uint64_t s, uint32_t d, uint32_t mid) {
  uint64_t nl = 0;
  for (uint64_t j = 0; j < s; j++)
#if MUT(29)
    if (t->q[(uint64_t)d * t->n + S[j]] <= mid) t->tmp[nl++] = S[j];
#else
    if (t->q[(uint64_t)d * t->n + S[j]] < mid) t->tmp[nl++] = S[j];
#endif
  uint64_t m = nl;
  for (uint64_t j = 0; j < s; j++)
#if MUT(29)
    if (!(t->q[(uint64_t)d * t->n + S[j]] <= mid)) t->tmp[m++] = S[j];
#else
    if (!(t->q[(uint64_t)d * t->n + S[j]] < mid)) t->tmp[m++] = S[j];
#endif
  memcpy(S, t->tmp, (size_t)s * sizeof(uint32_t));
  return nl;
}

/* The axis along which the members' codes spread widest (max - min), the
 * lowest axis on ties. */
static uint32_t widest_axis(const tree_t* t, const uint32_t* S, uint64_t s) {
  uint32_t best = 0;
  uint64_t wbest = 0;
  for (uint32_t d = 0; d < t->dims; d++) {
    const uint32_t* qd = t->q + (uint64_t)d * t->n;
    uint32_t lo = qd[S[0]], hi = qd[S[0]];
    for (uint64_t j = 1; j < s; j++) {
      if (qd[S[j]] < lo) lo = qd[S[j]];
      if (qd[S[j]] > hi) hi = qd[S[j]];
    }
    uint64_t w = (uint64_t)(hi - lo);
#if MUT(27)
    if (d == 0 || w < wbest) best = d, wbest = w; /* the narrowest instead */
#elif MUT(30)
    if (d == 0 || w >= wbest) best = d, wbest = w; /* ties to the last axis */
#else
    if (d == 0 || w > wbest) best = d, wbest = w;
#endif
  }
  return best;
}

/* Sec. 4.1 partition of the node order[start, start+s), depth-first, left
 * child first.  The rule (header byte 21) picks how a node splits:
 *   0  the paper's reading: halve until at most r particles, split at the
 *      median along the axes in turn (depth mod dims); the member of rank
 *      floor(s/2) in (q_d, index) order and everything after it form the
 *      right child, the median on the side of larger coordinates;
 *   1  as 0, along the axis of widest code extent among the node's members;
 *   2  ceil(n / r) leaves of floor or ceil of n / ceil(n / r) particles: leaf
 *      i holds the ranks floor(i n / b) .. floor((i + 1) n / b) - 1 of the
 *      tree order, b = ceil(n / r); a node holding leaves [i0, i1) gives its
 *      left child the first floor((i1 - i0) / 2) of them and splits at the
 *      matching rank, along the axes in turn;
 *   3  the midpoint (cell) split of the coders of Sec. 2.2: the root cell is
 *      the whole code grid [0, 2^G_d) per axis, a node of more than r
 *      particles halves its cell along the axes in turn, skipping axes whose
 *      cell is one code wide (a node whose cell is a single code stays one
 *      leaf), codes below the cell's midpoint go left, and an empty child
 *      is no leaf.
 * Every split is stable: both children keep ascending original index. */
static void kd_split(tree_t* t, uint64_t start, uint64_t s, uint32_t depth, node_t nd) {
  uint32_t* S = t->order + start;
  int leaf;
  if (t->rule == 2) {
    leaf = nd.i1 - nd.i0 <= 1;
  } else {
#if MUT(12)
    leaf = (s < t->r) || s <= 1;
#else
    leaf = (s <= t->r);
#endif
  }
#if MUT(3)
  uint32_t d = 0;
#else
  uint32_t d = depth % t->dims; /* round-robin split axis */
#endif
  if (!leaf && t->rule == 3) {
    uint32_t k = 0;
#if MUT(31)
    if (nd.lg[d] == 0) k = t->dims; /* stops at the first one-code-wide axis */
#endif
    while (k < t->dims && nd.lg[(d + k) % t->dims] == 0) k++;
    if (k == t->dims)
      leaf = 1; /* a single code: nothing to split */
    else
      d = (d + k) % t->dims;
  }
  if (leaf) {
    add_leaf(t, start, s);
    return;
  }
  node_t L = nd, R = nd;
  uint64_t nl;
  if (t->rule == 3) {
    uint32_t mid = nd.lo[d] + (1u << (nd.lg[d] - 1));
    nl = split_value(t, S, s, d, mid);
    L.lg[d] = R.lg[d] = nd.lg[d] - 1;
    R.lo[d] = mid;
    if (nl > 0) kd_split(t, start, nl, depth + 1, L);
    if (s - nl > 0) kd_split(t, start + nl, s - nl, depth + 1, R);
    return;
  }
  if (t->rule == 2) {
#if MUT(28)
    uint64_t im = nd.i0 + (nd.i1 - nd.i0 + 1) / 2; /* the left child takes the larger half */
#else
    uint64_t im = nd.i0 + (nd.i1 - nd.i0) / 2;
#endif
    uint64_t k = (im * t->n) / t->nb - (nd.i0 * t->n) / t->nb;
    nl = split_rank(t, S, s, d, k);
    L.i1 = im;
    R.i0 = im;
  } else {
    if (t->rule == 1) d = widest_axis(t, S, s);
    nl = split_rank(t, S, s, d, s / 2);
  }
  kd_split(t, start, nl, depth + 1, L);
  kd_split(t, start + nl, s - nl, depth + 1, R);
}

/* The same recursion on sizes only (children floor(s/2), ceil(s/2)): the leaf
 * sizes depend on (n, r) alone. */
static void size_leaves(uint64_t s, uint32_t r, uint32_t* out, uint64_t* k, uint64_t cap) {
  if (s <= r) {
    if (*k < cap) out[*k] = (uint32_t)s;
    (*k)++;
    return;
  }
  size_leaves(s / 2, r, out, k, cap);
  size_leaves(s - s / 2, r, out, k, cap);
}

static uint64_t count_leaves(uint64_t s, uint32_t r) {
  if (s <= r) return 1;
  return count_leaves(s / 2, r) + count_leaves(s - s / 2, r);
}

uint64_t bbxo_leaf_count(uint64_t n, uint32_t r) {
  if (n == 0 || r == 0) return 0;
  return count_leaves(n, r);
}

/* ------------------------------------------------------------------ bit box */

/* Sec. 4.1 bit box of one leaf: AABB, reference = member nearest the AABB
 * centre (squared Euclidean distance in code space, doubled to stay integral;
 * ties to the first member), then Eq. 2 per axis.  rule 1 (an ablation of
 * that choice): the reference is the member whose own Eq. 2 widths, taken
 * against the AABB, have the smallest sum (ties to the first member). */
static void bit_box(const uint32_t* q, uint64_t n, uint32_t dims, const uint32_t* mem,
                    uint64_t s, int rule, uint32_t* ref_out, uint32_t m_out[3]) {
  uint64_t qmin[3] = {0, 0, 0}, qmax[3] = {0, 0, 0};
  for (uint32_t d = 0; d < dims; d++) {
    qmin[d] = qmax[d] = q[(uint64_t)d * n + mem[0]];
    for (uint64_t j = 1; j < s; j++) {
      uint64_t v = q[(uint64_t)d * n + mem[j]];
      if (v < qmin[d]) qmin[d] = v;
      if (v > qmax[d]) qmax[d] = v;
    }
  }
  uint64_t best = UINT64_MAX, ref = 0;
  for (uint64_t j = 0; j < s; j++) {
    uint64_t dist = 0;
    for (uint32_t d = 0; d < dims; d++) {
      if (rule == 1) {
        uint64_t c = q[(uint64_t)d * n + mem[j]];
        dist += bbxo_bits_for_offset(c - qmin[d] > qmax[d] - c ? c - qmin[d] : qmax[d] - c);
        continue;
      }
      int64_t t = 2 * (int64_t)q[(uint64_t)d * n + mem[j]] - (int64_t)(qmin[d] + qmax[d]);
      dist += (uint64_t)(t * t);
    }
#if MUT(5)
    if (dist <= best) {
#else
    if (dist < best) {
#endif
      best = dist;
      ref = j;
    }
  }
#if MUT(4)
  ref = 0;
#endif
  *ref_out = (uint32_t)ref;
  for (uint32_t d = 0; d < 3; d++) m_out[d] = 0;
  for (uint32_t d = 0; d < dims; d++) {
    uint64_t c = q[(uint64_t)d * n + mem[ref]];
    uint64_t D = (c - qmin[d] > qmax[d] - c) ? c - qmin[d] : qmax[d] - c;
#if MUT(7)
    D = qmax[d] - qmin[d];
#endif
    m_out[d] = bbxo_bits_for_offset(D);
  }
}

/* ------------------------------------------------------------------ compress */

typedef struct {
  params_t p;
  uint32_t* q;     /* [dims][n] */
  uint32_t* order; /* [n] */
  uint64_t nleaves;
  uint32_t *leaf_start, *leaf_size, *leaf_ref;
  uint32_t* leaf_m; /* [nleaves][3] */
  uint64_t* leaf_bits;
  uint64_t meta_bits, payload_bits;
  int ref_mode; /* 0: reference stored as its code; 1: as its original coordinates */
  int split_rule; /* how nodes split (kd_split) */
  int lossless; /* the bound cannot be met by quantization: every coordinate stored as is */
} core_t;

static void core_free(core_t* c) {
  free(c->q);
  free(c->order);
  free(c->leaf_start);
  free(c->leaf_size);
  free(c->leaf_ref);
  free(c->leaf_m);
  free(c->leaf_bits);
  memset(c, 0, sizeof(*c));
}

static int check_args(uint64_t n, uint32_t dims, int dtype, int layout, double eb, int eb_mode,
                      uint32_t r, int ref_rule, int ref_mode) {
  if (ref_rule != 0 && ref_rule != 1) return BBXO_EINVAL;
  if (ref_mode != 0 && ref_mode != 1) return BBXO_EINVAL;
  if (dtype != 0 && dtype != 1) return BBXO_EINVAL;
  if (layout != 0 && layout != 1) return BBXO_EINVAL;
  if (eb_mode != 0 && eb_mode != 1) return BBXO_EINVAL;
  if (r == 0) return BBXO_EINVAL;
  if (!isfinite(eb) || !(eb > 0.0)) return BBXO_EINVAL;
  if (dims != 2 && dims != 3) return BBXO_EUNSUPPORTED;
  if (n >= ((uint64_t)1 << 32)) return BBXO_EUNSUPPORTED;
  return BBXO_OK;
}

/* ceil(n / r): the leaves of split rule 2 */
static uint64_t prop_leaf_count(uint64_t n, uint32_t r) {
#if MUT(32)
  return n / r ? n / r : 1;
#else
  return (n + r - 1) / r;
#endif
}

static int core_run(core_t* c, const void* pos, uint64_t n, uint32_t dims, int dtype, int layout,
                    double eb, int eb_mode, uint32_t r, int ref_rule, int ref_mode, int split_rule) {
  memset(c, 0, sizeof(*c));
  int st = check_args(n, dims, dtype, layout, eb, eb_mode, r, ref_rule, ref_mode);
  if (st) return st;
  if (split_rule < 0 || split_rule > 3) return BBXO_EINVAL;
  c->split_rule = split_rule;
  c->ref_mode = ref_mode;
  params_t* p = &c->p;
  p->n = n;
  p->dims = dims;
  p->dtype = dtype;
  p->eb_mode = eb_mode;
  p->r = r;
  p->eb_user = eb;
  p->mbits = dtype == 0 ? 5u : 6u; /* Sec. 4.2: 5 bits for M = 32, 6 for M = 64 */
  st = range_and_bound(pos, layout, p);
  /* Sec. 4.1: a coordinate that needs more than M bits is stored losslessly.
   * With codes on one global grid that happens to the whole set at once:
   * the bound is below what the input type resolves (eb_eff <= 0) or the
   * codes would need 30 bits or more; then every coordinate is stored as
   * its input bits (a version-3 stream) instead of failing. */
  if (st == BBXO_EBOUND) {
    c->lossless = 1;
    return BBXO_OK;
  }
  if (st) return st;
  if (n == 0) return BBXO_OK;

  /* leaves at most: rules 0 and 1 the count of the size recursion, rule 2
   * ceil(n / r), rule 3 one per particle (no leaf is empty) */
  uint64_t nl = split_rule <= 1 ? bbxo_leaf_count(n, r)
                                : (split_rule == 2 ? prop_leaf_count(n, r) : n);
  c->q = (uint32_t*)malloc((size_t)(n * dims) * sizeof(uint32_t));
  c->order = (uint32_t*)malloc((size_t)n * sizeof(uint32_t));
  c->leaf_start = (uint32_t*)malloc((size_t)nl * sizeof(uint32_t));
  c->leaf_size = (uint32_t*)malloc((size_t)nl * sizeof(uint32_t));
  c->leaf_ref = (uint32_t*)malloc((size_t)nl * sizeof(uint32_t));
  c->leaf_m = (uint32_t*)malloc((size_t)nl * 3 * sizeof(uint32_t));
  c->leaf_bits = (uint64_t*)malloc((size_t)nl * sizeof(uint64_t));
  uint64_t* keys = (uint64_t*)malloc((size_t)n * sizeof(uint64_t));
  uint32_t* tmp = (uint32_t*)malloc((size_t)n * sizeof(uint32_t));
  uint32_t* sz = (uint32_t*)malloc((size_t)nl * sizeof(uint32_t));
  if (!c->q || !c->order || !c->leaf_start || !c->leaf_size || !c->leaf_ref || !c->leaf_m ||
      !c->leaf_bits || !keys || !tmp || !sz) {
    free(keys);
    free(tmp);
    free(sz);
    return BBXO_ENOMEM;
  }

  /* Step 2: quantize every coordinate (codes of the whole set first). */
  for (uint32_t d = 0; d < dims; d++)
    for (uint64_t i = 0; i < n; i++)
      c->q[(uint64_t)d * n + i] =
          (uint32_t)quantize_real(coord(pos, p, layout, i, d), p->lo[d], p->inv_w);

  /* Step 3: k-d median partition. */
  for (uint64_t i = 0; i < n; i++) c->order[i] = (uint32_t)i;
  tree_t t;
  memset(&t, 0, sizeof(t));
  t.q = c->q;
  t.n = n;
  t.dims = dims;
  t.r = r;
  t.order = c->order;
  t.keys = keys;
  t.tmp = tmp;
  t.leaf_start = c->leaf_start;
  t.leaf_size = c->leaf_size;
  t.cap = nl;
  t.rule = split_rule;
  t.nb = prop_leaf_count(n, r);
  node_t root;
  memset(&root, 0, sizeof(root));
  root.i1 = t.nb;
  for (uint32_t d = 0; d < dims; d++) root.lg[d] = p->G[d];
  kd_split(&t, 0, n, 0, root);
  c->nleaves = t.nleaves;
  int same = !t.fail;
  if (split_rule <= 1) {
    /* the partition must reproduce the size-only recursion exactly */
    uint64_t k = 0;
    size_leaves(n, r, sz, &k, nl);
    same = same && k == nl && t.nleaves == nl;
    for (uint64_t i = 0; same && i < nl; i++) same = (sz[i] == c->leaf_size[i]);
  } else if (split_rule == 2) {
    same = same && t.nleaves == nl;
  }
  free(keys);
  free(tmp);
  free(sz);
  if (!same) return BBXO_ENOMEM; /* internal inconsistency: never expected */
  nl = c->nleaves;

  /* Step 4: bit box of every leaf; Step 5: section sizes.  The reference
   * field of a meta record holds its code (G_d bits per axis), or with
   * ref_mode 1 its original coordinate (M = 32 or 64 bits per axis). */
  uint32_t sumG = 0;
  for (uint32_t d = 0; d < dims; d++) sumG += ref_mode ? coord_bits(dtype) : p->G[d];
  c->meta_bits = nl * (uint64_t)(dims * p->mbits + sumG);
  c->payload_bits = 0;
  for (uint64_t i = 0; i < nl; i++) {
    uint32_t m[3];
    bit_box(c->q, n, dims, c->order + c->leaf_start[i], c->leaf_size[i], ref_rule,
            &c->leaf_ref[i], m);
    uint32_t sm = 0;
    for (uint32_t d = 0; d < 3; d++) {
      c->leaf_m[i * 3 + d] = m[d];
      sm += m[d];
    }
    c->leaf_bits[i] = (uint64_t)(c->leaf_size[i] - 1) * sm;
    c->payload_bits += c->leaf_bits[i];
  }
  return BBXO_OK;
}

static uint64_t words_bytes(uint64_t bits) { return ((bits + 63) / 64) * 8; }

uint64_t bbxo_compress_bound(uint64_t n, uint32_t dims, int dtype) {
  return bbxo_compress_bound_mode(n, dims, dtype, 0);
}

uint64_t bbxo_compress_bound_mode(uint64_t n, uint32_t dims, int dtype, int ref_mode) {
  uint64_t mbits = dtype == 1 ? 6 : 5;
  /* every particle is either a reference (dims*(mbits + G) <= dims*(mbits+30)
   * meta bits, or dims*(mbits + M) with ref_mode 1) or a member (dims*31
   * payload bits at most) */
  uint64_t ref = ref_mode ? coord_bits(dtype) : 30;
  uint64_t b = HEADER_BYTES + 16 + words_bytes(n * dims * (mbits + ref));
  uint64_t lossless = HEADER_BYTES + words_bytes(n * dims * coord_bits(dtype));
  return b > lossless ? b : lossless;
}

static void write_header(uint8_t* h, const core_t* c) {
  const params_t* p = &c->p;
  memset(h, 0, HEADER_BYTES);
  put_u32le(h + 0, MAGIC);
  put_u16le(h + 4, 1);
  h[6] = (uint8_t)p->dtype;
  h[7] = (uint8_t)p->dims;
  put_u64le(h + 8, p->n);
  put_u32le(h + 16, p->r);
  h[20] = (uint8_t)p->eb_mode;
  h[21] = (uint8_t)c->split_rule; /* how nodes split (kd_split); 0 in every version-1 stream */
  h[22] = (uint8_t)c->ref_mode; /* reference stored as its code (0) or coordinates (1) */
  h[23] = (uint8_t)p->mbits;
  put_f64le(h + 24, p->eb_user);
  put_f64le(h + 32, p->eb_abs);
  put_f64le(h + 40, p->eb_eff);
  put_f64le(h + 48, p->w);
  put_f64le(h + 56, p->inv_w);
  for (uint32_t d = 0; d < 3; d++) put_f64le(h + 64 + 8 * d, d < p->dims ? p->lo[d] : 0.0);
  for (uint32_t d = 0; d < 3; d++) h[88 + d] = (uint8_t)(d < p->dims ? p->G[d] : 0);
  put_u64le(h + 96, c->nleaves);
  put_u64le(h + 104, c->meta_bits);
  put_u64le(h + 112, c->payload_bits);
  put_u64le(h + 120, 0);
}

/* The lossless stream (version 3): the header with no grid (eb_eff, w,
 * inv_w, origin and G zero, no leaves, no meta section), then every input
 * coordinate's bits, M per value, particle by particle in input order (x, y,
 * z), zero-padded to 8 bytes.  Decoding returns the input exactly, in its
 * order (perm is the identity). */
static int write_lossless(const core_t* c, const void* pos, int layout, uint8_t* out,
                          uint64_t out_cap, uint64_t* out_size, uint32_t* perm) {
  const params_t* p = &c->p;
  const uint32_t M = coord_bits(p->dtype);
  const uint64_t bits = p->n * p->dims * M;
  const uint64_t total = HEADER_BYTES + words_bytes(bits);
  if (out_size) *out_size = total;
  if (total > out_cap) return BBXO_ENOSPC;
  memset(out, 0, (size_t)total);
  write_header(out, c);
  put_u16le(out + 4, 3);
  out[21] = 0; /* no partition */
  out[22] = 0; /* no reference field */
  for (int k = 40; k < 96; k++) out[k] = 0; /* eb_eff, w, inv_w, origin, G */
  put_u64le(out + 96, 0);
  put_u64le(out + 104, 0);
  put_u64le(out + 112, bits);
  uint8_t* pay = out + HEADER_BYTES;
  uint64_t at = 0;
  for (uint64_t i = 0; i < p->n; i++)
    for (uint32_t d = 0; d < p->dims; d++) {
#if MUT(26)
      put_bits(pay, at, coord_raw(pos, p, layout, i, p->dims - 1 - d), M); /* axes reversed */
#else
      put_bits(pay, at, coord_raw(pos, p, layout, i, d), M);
#endif
      at += M;
    }
  if (perm)
    for (uint64_t i = 0; i < p->n; i++) perm[i] = (uint32_t)i;
  return BBXO_OK;
}

int bbxo_compress(const void* pos, uint64_t n, uint32_t dims, int dtype, int layout, double eb,
                  int eb_mode, uint32_t r, uint8_t* out, uint64_t out_cap, uint64_t* out_size,
                  uint32_t* perm) {
  return bbxo_compress_ex(pos, n, dims, dtype, layout, eb, eb_mode, r, 0, 0, out, out_cap,
                          out_size, perm);
}

int bbxo_compress_ex(const void* pos, uint64_t n, uint32_t dims, int dtype, int layout, double eb,
                     int eb_mode, uint32_t r, int ref_rule, int ref_mode, uint8_t* out,
                     uint64_t out_cap, uint64_t* out_size, uint32_t* perm) {
  core_t c;
  int st = core_run(&c, pos, n, dims, dtype, layout, eb, eb_mode, r, ref_rule, ref_mode, 0);
  if (st || c.lossless) {
    if (!st) st = write_lossless(&c, pos, layout, out, out_cap, out_size, perm);
    core_free(&c);
    return st;
  }
  const params_t* p = &c.p;
  uint64_t mb = words_bytes(c.meta_bits), pb = words_bytes(c.payload_bits);
  uint64_t total = HEADER_BYTES + mb + pb;
  if (out_size) *out_size = total;
  if (total > out_cap) {
    core_free(&c);
    return BBXO_ENOSPC;
  }
  memset(out, 0, (size_t)total);
  write_header(out, &c);
  uint8_t* meta = out + HEADER_BYTES;
  uint8_t* pay = meta + mb;
  uint64_t mpos = 0, ppos = 0;
  for (uint64_t i = 0; i < c.nleaves; i++) {
    const uint32_t* mem = c.order + c.leaf_start[i];
    uint32_t s = c.leaf_size[i], ref = c.leaf_ref[i];
    const uint32_t* m = c.leaf_m + 3 * i;
    /* meta record: widths m_d (mbits each), then the reference's codes, or
     * with ref_mode 1 the bits of its original coordinates (Sec. 4.2) */
    for (uint32_t d = 0; d < p->dims; d++) put_bits(meta, mpos, m[d], p->mbits), mpos += p->mbits;
    for (uint32_t d = 0; d < p->dims; d++) {
      if (ref_mode) {
#if MUT(16)
        uint32_t src = mem[0];
#else
        uint32_t src = mem[ref];
#endif
        put_bits(meta, mpos, coord_raw(pos, p, layout, src, d), coord_bits(dtype));
        mpos += coord_bits(dtype);
      } else {
        put_bits(meta, mpos, c.q[(uint64_t)d * n + mem[ref]], p->G[d]);
        mpos += p->G[d];
      }
    }
    /* payload: every other member in leaf order, codes o + 2^(m-1) per axis */
    for (uint32_t jj = 0; jj < s; jj++) {
#if MUT(13)
      uint32_t j = s - 1 - jj;
#else
      uint32_t j = jj;
#endif
      if (j == ref) continue;
      for (uint32_t dd = 0; dd < p->dims; dd++) {
#if MUT(8)
        uint32_t d = p->dims - 1 - dd;
#else
        uint32_t d = dd;
#endif
        if (m[d] == 0) continue;
        int64_t o = (int64_t)c.q[(uint64_t)d * n + mem[j]] - (int64_t)c.q[(uint64_t)d * n + mem[ref]];
        uint64_t u = (uint64_t)(o + ((int64_t)1 << (m[d] - 1)));
        put_bits(pay, ppos, u, m[d]);
        ppos += m[d];
      }
    }
    if (perm) {
      uint64_t slot = c.leaf_start[i];
      perm[slot++] = mem[ref];
      for (uint32_t j = 0; j < s; j++)
        if (j != ref) perm[slot++] = mem[j];
    }
  }
  core_free(&c);
  return BBXO_OK;
}

int bbxo_stages(const void* pos, uint64_t n, uint32_t dims, int dtype, int layout, double eb,
                int eb_mode, uint32_t r, uint32_t* q, uint32_t* order, uint64_t max_leaves,
                uint32_t* leaf_start, uint32_t* leaf_size, uint32_t* leaf_ref, uint8_t* leaf_m,
                uint64_t* leaf_bits, double* scal) {
  return bbxo_stages_ex(pos, n, dims, dtype, layout, eb, eb_mode, r, 0, q, order, max_leaves,
                        leaf_start, leaf_size, leaf_ref, leaf_m, leaf_bits, scal);
}

int bbxo_stages_ex(const void* pos, uint64_t n, uint32_t dims, int dtype, int layout, double eb,
                   int eb_mode, uint32_t r, int ref_rule, uint32_t* q, uint32_t* order,
                   uint64_t max_leaves, uint32_t* leaf_start, uint32_t* leaf_size,
                   uint32_t* leaf_ref, uint8_t* leaf_m, uint64_t* leaf_bits, double* scal) {
  core_t c;
  int st = core_run(&c, pos, n, dims, dtype, layout, eb, eb_mode, r, ref_rule, 0, 0);
  if (!st && c.lossless) st = BBXO_EBOUND; /* no partition or bit boxes to dump */
  if (st) {
    core_free(&c);
    return st;
  }
  if (scal) {
    scal[0] = c.p.eb_abs;
    scal[1] = c.p.eb_eff;
    scal[2] = c.p.w;
    scal[3] = c.p.inv_w;
    for (int d = 0; d < 3; d++) {
      scal[4 + d] = c.p.lo[d];
      scal[7 + d] = c.p.hi[d];
      scal[10 + d] = (double)c.p.G[d];
    }
    scal[13] = (double)c.nleaves;
    scal[14] = (double)c.meta_bits;
    scal[15] = (double)c.payload_bits;
  }
  if (n > 0) {
    if (q) memcpy(q, c.q, (size_t)(n * dims) * sizeof(uint32_t));
    if (order) memcpy(order, c.order, (size_t)n * sizeof(uint32_t));
  }
  uint64_t L = c.nleaves < max_leaves ? c.nleaves : max_leaves;
  for (uint64_t i = 0; i < L; i++) {
    if (leaf_start) leaf_start[i] = c.leaf_start[i];
    if (leaf_size) leaf_size[i] = c.leaf_size[i];
    if (leaf_ref) leaf_ref[i] = c.leaf_ref[i];
    if (leaf_m)
      for (int d = 0; d < 3; d++) leaf_m[i * 3 + d] = (uint8_t)c.leaf_m[i * 3 + d];
    if (leaf_bits) leaf_bits[i] = c.leaf_bits[i];
  }
  core_free(&c);
  return BBXO_OK;
}

/* ------------------------------------------------------------------ bit box reduction */

/* Sec. 4.1 "Bit box reduction and bit box intersection update", the while
 * loop of Alg. 1, on the leaves (subregions) of the partition above:
 *   - a leaf's bit box is its reference's codes c_d and widths m_d; in code
 *     space it holds exactly the codes q with |q_d - c_d| <= R(m_d), R(m) =
 *     2^(m-1) - 1 (R(0) = 0): the offsets its widths can encode (Eq. 1/3);
 *   - repeatedly pop the remaining leaf with the smallest key (key_rule 0:
 *     the sum of widths sum_d m_d, as the text says; key_rule 1: the sum of
 *     box lengths sum_d (2^m_d - 1) in bins, as the figure caption says),
 *     ties to the first leaf in depth-first order;
 *   - its sequence holds the centre (its reference), its other remaining
 *     members in ascending index, then the common particles: the remaining
 *     members of every other remaining leaf whose bit box intersects the
 *     popped one and that lie inside the popped box, leaf by leaf in
 *     depth-first order, each leaf's in ascending index;
 *   - every leaf that lost particles gets its bit box again from what it
 *     keeps (AABB, member nearest the AABB centre, Eq. 2); a leaf left empty
 *     vanishes without a sequence.
 * The loop ends when no particle remains. */
typedef struct {
  uint32_t ref;  /* source index of the current reference */
  uint32_t m[3];
  uint32_t cnt;  /* remaining members */
  int live;      /* not popped and not empty */
} rbox_t;

static uint32_t box_reach(uint32_t m) { return m ? ((1u << (m - 1)) - 1u) : 0u; }

static uint64_t box_key(const rbox_t* b, uint32_t dims, int key_rule) {
  uint64_t k = 0;
  for (uint32_t d = 0; d < dims; d++) {
#if MUT(21)
    k += key_rule == 0 ? ((1ull << b->m[d]) - 1) : b->m[d];
#else
    k += key_rule == 0 ? b->m[d] : ((1ull << b->m[d]) - 1);
#endif
  }
  return k;
}

static int boxes_meet(const uint32_t* q, uint64_t n, uint32_t dims, const rbox_t* a,
                      const rbox_t* b) {
  for (uint32_t d = 0; d < dims; d++) {
    int64_t ca = q[(uint64_t)d * n + a->ref], cb = q[(uint64_t)d * n + b->ref];
    int64_t gap = ca > cb ? ca - cb : cb - ca;
    if (gap > (int64_t)box_reach(a->m[d]) + (int64_t)box_reach(b->m[d])) return 0;
  }
  return 1;
}

static int box_holds(const uint32_t* q, uint64_t n, uint32_t dims, const rbox_t* a, uint32_t i) {
  for (uint32_t d = 0; d < dims; d++) {
    int64_t o = (int64_t)q[(uint64_t)d * n + i] - (int64_t)q[(uint64_t)d * n + a->ref];
    if ((o < 0 ? -o : o) > (int64_t)box_reach(a->m[d])) return 0;
  }
  return 1;
}

typedef struct {
  uint64_t nseq;
  uint32_t* seq_center; /* [nseq] source index */
  uint32_t* seq_m;      /* [nseq][3] */
  uint32_t* seq_count;  /* [nseq] particles besides the centre */
  uint32_t* slot_src;   /* [n] source index per output slot */
} reduced_t;

static void reduced_free(reduced_t* r) {
  free(r->seq_center);
  free(r->seq_m);
  free(r->seq_count);
  free(r->slot_src);
  memset(r, 0, sizeof(*r));
}

static int reduce_boxes(const core_t* c, int key_rule, reduced_t* out) {
  const uint64_t n = c->p.n, nl = c->nleaves;
  const uint32_t dims = c->p.dims;
  memset(out, 0, sizeof(*out));
  rbox_t* box = (rbox_t*)calloc((size_t)(nl ? nl : 1), sizeof(rbox_t));
  uint8_t* taken = (uint8_t*)calloc((size_t)(n ? n : 1), 1);
  uint64_t big = 1;
  for (uint64_t b = 0; b < nl; b++)
    if (c->leaf_size[b] > big) big = c->leaf_size[b];
  uint32_t* mem = (uint32_t*)malloc((size_t)(big + 1) * sizeof(uint32_t));
  out->seq_center = (uint32_t*)malloc((size_t)(nl ? nl : 1) * sizeof(uint32_t));
  out->seq_m = (uint32_t*)malloc((size_t)(nl ? nl : 1) * 3 * sizeof(uint32_t));
  out->seq_count = (uint32_t*)malloc((size_t)(nl ? nl : 1) * sizeof(uint32_t));
  out->slot_src = (uint32_t*)malloc((size_t)(n ? n : 1) * sizeof(uint32_t));
  if (!box || !taken || !mem || !out->seq_center || !out->seq_m || !out->seq_count ||
      !out->slot_src) {
    free(box), free(taken), free(mem);
    reduced_free(out);
    return BBXO_ENOMEM;
  }
  /* the bit boxes of the partition's leaves (Step 4) */
  for (uint64_t b = 0; b < nl; b++) {
    box[b].ref = c->order[c->leaf_start[b] + c->leaf_ref[b]];
    for (int d = 0; d < 3; d++) box[b].m[d] = c->leaf_m[3 * b + d];
    box[b].cnt = c->leaf_size[b];
    box[b].live = 1;
  }
  uint64_t slot = 0, left = n;
  while (left > 0) {
    /* the remaining box with the smallest key, first in leaf order on ties */
    uint64_t cur = nl;
    uint64_t best = 0;
    for (uint64_t b = 0; b < nl; b++) {
      if (!box[b].live) continue;
      uint64_t k = box_key(&box[b], dims, key_rule);
#if MUT(22)
      if (cur == nl || k <= best) cur = b, best = k;
#else
      if (cur == nl || k < best) cur = b, best = k;
#endif
    }
    if (cur == nl) break; /* never: particles remain only in live boxes */
    rbox_t* B = &box[cur];
    uint64_t s = out->nseq++;
    out->seq_center[s] = B->ref;
    for (int d = 0; d < 3; d++) out->seq_m[3 * s + d] = B->m[d];
    uint64_t first = slot;
    out->slot_src[slot++] = B->ref;
    taken[B->ref] = 1;
    /* its other remaining members, ascending index */
    const uint32_t* L = c->order + c->leaf_start[cur];
    for (uint32_t j = 0; j < c->leaf_size[cur]; j++)
      if (!taken[L[j]]) {
        taken[L[j]] = 1;
        out->slot_src[slot++] = L[j];
      }
    /* common particles of the intersecting boxes, leaf by leaf */
#if MUT(25)
    for (uint64_t bb = nl; bb-- > 0;) {
      uint64_t b = bb;
#else
    for (uint64_t b = 0; b < nl; b++) {
#endif
      if (b == cur || !box[b].live || !boxes_meet(c->q, n, dims, B, &box[b])) continue;
#if MUT(24)
      continue;
#endif
      const uint32_t* M = c->order + c->leaf_start[b];
      uint32_t lost = 0, kept = 0;
      for (uint32_t j = 0; j < c->leaf_size[b]; j++) {
        uint32_t i = M[j];
        if (taken[i]) continue;
        if (box_holds(c->q, n, dims, B, i)) {
          taken[i] = 1;
          out->slot_src[slot++] = i;
          lost++;
        } else {
          mem[kept++] = i;
        }
      }
      if (lost == 0) continue;
      box[b].cnt = kept;
      if (kept == 0) {
        box[b].live = 0; /* empty: vanishes */
        continue;
      }
#if !MUT(23)
      uint32_t ref = 0, m[3];
      bit_box(c->q, n, dims, mem, kept, 0, &ref, m);
      box[b].ref = mem[ref];
      for (int d = 0; d < 3; d++) box[b].m[d] = m[d];
#endif
    }
    out->seq_count[s] = (uint32_t)(slot - first - 1);
    left -= slot - first;
    B->live = 0;
    B->cnt = 0;
  }
  free(box), free(taken), free(mem);
  if (slot != n) {
    reduced_free(out);
    return BBXO_ENOMEM; /* internal inconsistency: never expected */
  }
  return BBXO_OK;
}

/* Every leaf as one sequence, in leaf order: its reference, then its other
 * members in ascending index (the stream of a partition without the
 * reduction). */
static int leaf_sequences(const core_t* c, reduced_t* out) {
  const uint64_t n = c->p.n, nl = c->nleaves;
  memset(out, 0, sizeof(*out));
  out->seq_center = (uint32_t*)malloc((size_t)(nl ? nl : 1) * sizeof(uint32_t));
  out->seq_m = (uint32_t*)malloc((size_t)(nl ? nl : 1) * 3 * sizeof(uint32_t));
  out->seq_count = (uint32_t*)malloc((size_t)(nl ? nl : 1) * sizeof(uint32_t));
  out->slot_src = (uint32_t*)malloc((size_t)(n ? n : 1) * sizeof(uint32_t));
  if (!out->seq_center || !out->seq_m || !out->seq_count || !out->slot_src) {
    reduced_free(out);
    return BBXO_ENOMEM;
  }
  uint64_t slot = 0;
  for (uint64_t b = 0; b < nl; b++) {
    const uint32_t* L = c->order + c->leaf_start[b];
    out->seq_center[b] = L[c->leaf_ref[b]];
    for (int d = 0; d < 3; d++) out->seq_m[3 * b + d] = c->leaf_m[3 * b + d];
    out->seq_count[b] = c->leaf_size[b] - 1;
    out->slot_src[slot++] = L[c->leaf_ref[b]];
    for (uint32_t j = 0; j < c->leaf_size[b]; j++)
      if (j != c->leaf_ref[b]) out->slot_src[slot++] = L[j];
  }
  out->nseq = nl;
  return BBXO_OK;
}

/* Stream of sequences (version 2 of the format): the v1 header with version
 * 2, the split rule in byte 21, the partition's leaf count and the sequence
 * count in the last field; a meta record per sequence (widths m_d in mbits
 * bits, the centre's codes in G_d bits, then the number of other particles
 * in 32 bits: the end mark of Sec. 4.2 turned into a count); the payload
 * holds each sequence's particles in order, per axis q_d - c_d + 2^(m_d - 1)
 * in m_d bits. */
static int write_sequences(core_t* c, const reduced_t* R, uint8_t* out, uint64_t out_cap,
                           uint64_t* out_size, uint32_t* perm) {
  const params_t* p = &c->p;
  const uint64_t n = p->n;
  const uint32_t dims = p->dims;
  uint32_t sumG = 0;
  for (uint32_t d = 0; d < dims; d++) sumG += p->G[d];
  uint64_t meta_bits = R->nseq * (uint64_t)(dims * p->mbits + sumG + 32), payload_bits = 0;
  for (uint64_t s = 0; s < R->nseq; s++) {
    uint32_t sm = 0;
    for (uint32_t d = 0; d < dims; d++) sm += R->seq_m[3 * s + d];
    payload_bits += (uint64_t)R->seq_count[s] * sm;
  }
  uint64_t mb = words_bytes(meta_bits), pb = words_bytes(payload_bits);
  uint64_t total = HEADER_BYTES + mb + pb;
  if (out_size) *out_size = total;
  if (total > out_cap) return BBXO_ENOSPC;
  memset(out, 0, (size_t)total);
  c->meta_bits = meta_bits;
  c->payload_bits = payload_bits;
  write_header(out, c);
  put_u16le(out + 4, 2);
  put_u64le(out + 120, R->nseq);
  uint8_t* meta = out + HEADER_BYTES;
  uint8_t* pay = meta + mb;
  uint64_t mpos = 0, ppos = 0, slot = 0;
  for (uint64_t s = 0; s < R->nseq; s++) {
    const uint32_t* m = R->seq_m + 3 * s;
    uint32_t ctr = R->seq_center[s];
    for (uint32_t d = 0; d < dims; d++) put_bits(meta, mpos, m[d], p->mbits), mpos += p->mbits;
    for (uint32_t d = 0; d < dims; d++)
      put_bits(meta, mpos, c->q[(uint64_t)d * n + ctr], p->G[d]), mpos += p->G[d];
    put_bits(meta, mpos, R->seq_count[s], 32), mpos += 32;
    slot++; /* the centre */
    for (uint32_t j = 0; j < R->seq_count[s]; j++, slot++) {
      uint32_t i = R->slot_src[slot];
      for (uint32_t d = 0; d < dims; d++) {
        if (m[d] == 0) continue;
        int64_t o = (int64_t)c->q[(uint64_t)d * n + i] - (int64_t)c->q[(uint64_t)d * n + ctr];
        put_bits(pay, ppos, (uint64_t)(o + ((int64_t)1 << (m[d] - 1))), m[d]);
        ppos += m[d];
      }
    }
  }
  if (perm && n) memcpy(perm, R->slot_src, (size_t)n * sizeof(uint32_t));
  return BBXO_OK;
}

int bbxo_compress_split(const void* pos, uint64_t n, uint32_t dims, int dtype, int layout,
                        double eb, int eb_mode, uint32_t r, int split_rule, int ref_rule,
                        int reduce, uint8_t* out, uint64_t out_cap, uint64_t* out_size,
                        uint32_t* perm) {
  if (reduce < 0 || reduce > 2 || split_rule < 0 || split_rule > 3) return BBXO_EINVAL;
  if (split_rule == 0 && reduce == 0)
    return bbxo_compress_ex(pos, n, dims, dtype, layout, eb, eb_mode, r, ref_rule, 0, out, out_cap,
                            out_size, perm);
  core_t c;
  int st = core_run(&c, pos, n, dims, dtype, layout, eb, eb_mode, r, ref_rule, 0, split_rule);
  if (st || c.lossless) {
    if (!st) st = write_lossless(&c, pos, layout, out, out_cap, out_size, perm);
    core_free(&c);
    return st;
  }
  reduced_t R;
  memset(&R, 0, sizeof(R));
  if (n > 0) {
    st = reduce ? reduce_boxes(&c, reduce - 1, &R) : leaf_sequences(&c, &R);
    if (st) {
      core_free(&c);
      return st;
    }
  }
  st = write_sequences(&c, &R, out, out_cap, out_size, perm);
  reduced_free(&R);
  core_free(&c);
  return st;
}

int bbxo_compress_reduced(const void* pos, uint64_t n, uint32_t dims, int dtype, int layout,
                          double eb, int eb_mode, uint32_t r, int key_rule, uint8_t* out,
                          uint64_t out_cap, uint64_t* out_size, uint32_t* perm) {
  if (key_rule != 0 && key_rule != 1) return BBXO_EINVAL;
  return bbxo_compress_split(pos, n, dims, dtype, layout, eb, eb_mode, r, 0, 0, key_rule + 1, out,
                             out_cap, out_size, perm);
}

/* ------------------------------------------------------------------ decompress */

static int decompress_reduced(const uint8_t* s, uint64_t size, void* pos, uint64_t pos_cap_bytes,
                              int layout);
static int decompress_lossless(const uint8_t* s, uint64_t size, void* pos, uint64_t pos_cap_bytes,
                               int layout);

int bbxo_decompress(const uint8_t* s, uint64_t size, void* pos, uint64_t pos_cap_bytes,
                    int layout) {
  if (layout != 0 && layout != 1) return BBXO_EINVAL;
  if (!s || size < HEADER_BYTES) return BBXO_ECORRUPT;
  if (get_u32le(s) == MAGIC && get_u16le(s + 4) == 2)
    return decompress_reduced(s, size, pos, pos_cap_bytes, layout);
  if (get_u32le(s) == MAGIC && get_u16le(s + 4) == 3)
    return decompress_lossless(s, size, pos, pos_cap_bytes, layout);
  if (get_u32le(s) != MAGIC || get_u16le(s + 4) != 1) return BBXO_ECORRUPT;
  int dtype = s[6];
  uint32_t dims = s[7];
  uint64_t n = get_u64le(s + 8);
  uint32_t r = get_u32le(s + 16);
  uint32_t eb_mode = s[20], mbits = s[23];
  if (dtype > 1 || (dims != 2 && dims != 3) || eb_mode > 1 || s[21] != 0 || s[22] > 1)
    return BBXO_ECORRUPT;
  int ref_mode = s[22];
  uint32_t M = coord_bits(dtype);
  if (mbits != (dtype == 0 ? 5u : 6u) || r == 0 || n >= ((uint64_t)1 << 32)) return BBXO_ECORRUPT;
  double w = get_f64le(s + 48), inv_w = get_f64le(s + 56);
  double origin[3];
  uint32_t G[3], sumG = 0;
  for (uint32_t d = 0; d < 3; d++) {
    origin[d] = get_f64le(s + 64 + 8 * d);
    G[d] = s[88 + d];
    if (d >= dims && (G[d] != 0 || origin[d] != 0.0)) return BBXO_ECORRUPT;
    if (G[d] > 30 || !isfinite(origin[d])) return BBXO_ECORRUPT;
    sumG += G[d];
  }
  if (!isfinite(w) || w < 0.0 || !isfinite(inv_w) || inv_w < 0.0) return BBXO_ECORRUPT;
  for (int k = 91; k < 96; k++)
    if (s[k] != 0) return BBXO_ECORRUPT;
  uint64_t nl = get_u64le(s + 96), meta_bits = get_u64le(s + 104), payload_bits = get_u64le(s + 112);
  if (get_u64le(s + 120) != 0) return BBXO_ECORRUPT;
  if (nl != bbxo_leaf_count(n, r)) return BBXO_ECORRUPT;
  if (meta_bits != nl * (uint64_t)(dims * mbits + (ref_mode ? dims * M : sumG)))
    return BBXO_ECORRUPT;
  if (payload_bits > n * (uint64_t)dims * 31u) return BBXO_ECORRUPT;
  uint64_t mb = words_bytes(meta_bits), pb = words_bytes(payload_bits);
  if (size < HEADER_BYTES + mb + pb) return BBXO_ECORRUPT;
  uint64_t esz = dtype == 0 ? 4 : 8;
  if (pos_cap_bytes < n * dims * esz) return BBXO_ENOSPC;
  if (n == 0) return BBXO_OK;

  const uint8_t* meta = s + HEADER_BYTES;
  const uint8_t* pay = meta + mb;
  uint32_t* sizes = (uint32_t*)malloc((size_t)nl * sizeof(uint32_t));
  uint32_t* codes = (uint32_t*)malloc((size_t)(n * dims) * sizeof(uint32_t)); /* [slot][d] */
  uint64_t* rraw = (uint64_t*)malloc((size_t)(nl * dims) * sizeof(uint64_t)); /* ref_mode 1 */
  if (!sizes || !codes || !rraw) {
    free(sizes);
    free(codes);
    free(rraw);
    return BBXO_ENOMEM;
  }
  uint64_t k = 0;
  size_leaves(n, r, sizes, &k, nl);
  int st = BBXO_OK;
  uint64_t mpos = 0, ppos = 0, slot = 0;
  for (uint64_t i = 0; i < nl && st == BBXO_OK; i++) {
    uint32_t m[3] = {0, 0, 0};
    uint64_t qref[3] = {0, 0, 0};
    for (uint32_t d = 0; d < dims; d++) {
      m[d] = (uint32_t)get_bits(meta, mpos, mbits);
      mpos += mbits;
      if (m[d] == 1 || m[d] > 31 || m[d] > G[d] + 1) st = BBXO_ECORRUPT;
    }
    for (uint32_t d = 0; d < dims; d++) {
      if (ref_mode) {
        /* the stored coordinate; its code is what the encoder's quantization
         * gave it (same origin, same 1/w, same FP64 operations) */
        uint64_t raw = get_bits(meta, mpos, M);
        mpos += M;
        rraw[i * dims + d] = raw;
        double x;
        if (dtype == 0) {
          uint32_t u32 = (uint32_t)raw;
          float f;
          memcpy(&f, &u32, 4);
          x = (double)f;
        } else {
          memcpy(&x, &raw, 8);
        }
        double qd = isfinite(x) ? quantize_real(x, origin[d], inv_w) : -1.0;
        if (!(qd >= 0.0 && qd < (double)((uint64_t)1 << G[d]))) st = BBXO_ECORRUPT;
        qref[d] = st ? 0 : (uint64_t)qd;
      } else {
        qref[d] = get_bits(meta, mpos, G[d]);
        mpos += G[d];
      }
    }
    if (st) break;
    uint32_t sm = 0;
    for (uint32_t d = 0; d < dims; d++) sm += m[d];
    if (ppos + (uint64_t)(sizes[i] - 1) * sm > payload_bits) {
      st = BBXO_ECORRUPT;
      break;
    }
    for (uint32_t d = 0; d < dims; d++) codes[slot * dims + d] = (uint32_t)qref[d];
    slot++;
    for (uint32_t j = 1; j < sizes[i] && st == BBXO_OK; j++, slot++) {
      for (uint32_t d = 0; d < dims; d++) {
        int64_t qv = (int64_t)qref[d];
        if (m[d] > 0) {
          uint64_t u = get_bits(pay, ppos, m[d]);
          ppos += m[d];
          if (u == 0) st = BBXO_ECORRUPT; /* code 0 is never emitted */
          qv = (int64_t)qref[d] + (int64_t)u - ((int64_t)1 << (m[d] - 1));
        }
        if (qv < 0 || qv >= ((int64_t)1 << G[d])) st = BBXO_ECORRUPT;
        codes[slot * dims + d] = (uint32_t)qv;
      }
    }
  }
  if (st == BBXO_OK && ppos != payload_bits) st = BBXO_ECORRUPT;
  if (st == BBXO_OK) {
    /* Sec. 3 dequantization: the bin centre origin + q*w (multiply, then add,
     * each rounded), then rounded to the stream's type. */
    for (uint64_t i = 0; i < n; i++)
      for (uint32_t d = 0; d < dims; d++) {
        double qw = (double)codes[i * dims + d] * w;
#if MUT(11)
        double v = origin[d] + qw + 0.5 * w;
#else
        double v = origin[d] + qw;
#endif
        uint64_t kk = (layout == 0) ? i * dims + d : (uint64_t)d * n + i;
        if (dtype == 0)
          ((float*)pos)[kk] = (float)v;
        else
          ((double*)pos)[kk] = v;
      }
#if !MUT(17)
    /* ref_mode 1: each leaf's reference (its first slot) is its stored
     * coordinate, exactly */
    for (uint64_t i = 0, slot0 = 0; ref_mode && i < nl; slot0 += sizes[i], i++)
      for (uint32_t d = 0; d < dims; d++) {
        uint64_t kk = (layout == 0) ? slot0 * dims + d : (uint64_t)d * n + slot0;
        uint64_t raw = rraw[i * dims + d];
        if (dtype == 0) {
          uint32_t u32 = (uint32_t)raw;
          memcpy((float*)pos + kk, &u32, 4);
        } else {
          memcpy((double*)pos + kk, &raw, 8);
        }
      }
#endif
  }
  free(sizes);
  free(codes);
  free(rraw);
  return st;
}

/* Decoder of the reduced stream (version 2): sequences in stored order; in
 * each the centre, then its other particles in stored order. */
static int decompress_reduced(const uint8_t* s, uint64_t size, void* pos, uint64_t pos_cap_bytes,
                              int layout) {
  int dtype = s[6];
  uint32_t dims = s[7];
  uint64_t n = get_u64le(s + 8);
  uint32_t r = get_u32le(s + 16);
  uint32_t eb_mode = s[20], mbits = s[23];
  const uint32_t rule = s[21];
  if (dtype > 1 || (dims != 2 && dims != 3) || eb_mode > 1 || rule > 3 || s[22] != 0)
    return BBXO_ECORRUPT;
  if (mbits != (dtype == 0 ? 5u : 6u) || r == 0 || n >= ((uint64_t)1 << 32)) return BBXO_ECORRUPT;
  double w = get_f64le(s + 48), inv_w = get_f64le(s + 56);
  double origin[3];
  uint32_t G[3], sumG = 0;
  for (uint32_t d = 0; d < 3; d++) {
    origin[d] = get_f64le(s + 64 + 8 * d);
    G[d] = s[88 + d];
    if (d >= dims && (G[d] != 0 || origin[d] != 0.0)) return BBXO_ECORRUPT;
    if (G[d] > 30 || !isfinite(origin[d])) return BBXO_ECORRUPT;
    sumG += G[d];
  }
  if (!isfinite(w) || w < 0.0 || !isfinite(inv_w) || inv_w < 0.0) return BBXO_ECORRUPT;
  for (int k = 91; k < 96; k++)
    if (s[k] != 0) return BBXO_ECORRUPT;
  uint64_t nl = get_u64le(s + 96), meta_bits = get_u64le(s + 104), payload_bits = get_u64le(s + 112);
  uint64_t nseq = get_u64le(s + 120);
  /* the partition's leaf count: fixed by (n, r) for rules 0 to 2, at most
   * one per particle for rule 3 */
  uint64_t want = rule <= 1 ? bbxo_leaf_count(n, r) : prop_leaf_count(n, r);
  if (rule == 3 ? (nl > n || (n > 0 && nl == 0)) : nl != want) return BBXO_ECORRUPT;
  if (nseq > nl || (n > 0 && nseq == 0)) return BBXO_ECORRUPT;
  if (meta_bits != nseq * (uint64_t)(dims * mbits + sumG + 32)) return BBXO_ECORRUPT;
  if (payload_bits > n * (uint64_t)dims * 31u) return BBXO_ECORRUPT;
  uint64_t mb = words_bytes(meta_bits), pb = words_bytes(payload_bits);
  if (size < HEADER_BYTES + mb + pb) return BBXO_ECORRUPT;
  uint64_t esz = dtype == 0 ? 4 : 8;
  if (pos_cap_bytes < n * dims * esz) return BBXO_ENOSPC;
  if (n == 0) return BBXO_OK;
  const uint8_t* meta = s + HEADER_BYTES;
  const uint8_t* pay = meta + mb;
  uint32_t* codes = (uint32_t*)malloc((size_t)(n * dims) * sizeof(uint32_t));
  if (!codes) return BBXO_ENOMEM;
  int st = BBXO_OK;
  uint64_t mpos = 0, ppos = 0, slot = 0;
  for (uint64_t q = 0; q < nseq && st == BBXO_OK; q++) {
    uint32_t m[3] = {0, 0, 0}, sm = 0;
    int64_t ctr[3] = {0, 0, 0};
    for (uint32_t d = 0; d < dims; d++) {
      m[d] = (uint32_t)get_bits(meta, mpos, mbits);
      mpos += mbits;
      if (m[d] == 1 || m[d] > 31 || m[d] > G[d] + 1) st = BBXO_ECORRUPT;
      sm += m[d];
    }
    for (uint32_t d = 0; d < dims; d++) ctr[d] = (int64_t)get_bits(meta, mpos, G[d]), mpos += G[d];
    uint64_t cnt = get_bits(meta, mpos, 32);
    mpos += 32;
    if (st || slot + 1 + cnt > n || ppos + cnt * sm > payload_bits) {
      st = BBXO_ECORRUPT;
      break;
    }
    for (uint32_t d = 0; d < dims; d++) codes[slot * dims + d] = (uint32_t)ctr[d];
    slot++;
    for (uint64_t j = 0; j < cnt && st == BBXO_OK; j++, slot++)
      for (uint32_t d = 0; d < dims; d++) {
        int64_t qv = ctr[d];
        if (m[d] > 0) {
          uint64_t u = get_bits(pay, ppos, m[d]);
          ppos += m[d];
          if (u == 0) st = BBXO_ECORRUPT;
          qv = ctr[d] + (int64_t)u - ((int64_t)1 << (m[d] - 1));
        }
        if (qv < 0 || qv >= ((int64_t)1 << G[d])) st = BBXO_ECORRUPT;
        codes[slot * dims + d] = (uint32_t)qv;
      }
  }
  if (st == BBXO_OK && (slot != n || ppos != payload_bits)) st = BBXO_ECORRUPT;
  if (st == BBXO_OK)
    for (uint64_t i = 0; i < n; i++)
      for (uint32_t d = 0; d < dims; d++) {
        double v = origin[d] + (double)codes[i * dims + d] * w;
        uint64_t kk = (layout == 0) ? i * dims + d : (uint64_t)d * n + i;
        if (dtype == 0)
          ((float*)pos)[kk] = (float)v;
        else
          ((double*)pos)[kk] = v;
      }
  free(codes);
  return st;
}

/* Decoder of the lossless stream (version 3). */
static int decompress_lossless(const uint8_t* s, uint64_t size, void* pos, uint64_t pos_cap_bytes,
                               int layout) {
  int dtype = s[6];
  uint32_t dims = s[7];
  uint64_t n = get_u64le(s + 8);
  if (dtype > 1 || (dims != 2 && dims != 3) || s[20] > 1 || s[21] != 0 || s[22] != 0 ||
      s[23] != (dtype == 0 ? 5u : 6u) || get_u32le(s + 16) == 0 || n >= ((uint64_t)1 << 32))
    return BBXO_ECORRUPT;
  for (int k = 40; k < 104; k++)
    if (s[k] != 0) return BBXO_ECORRUPT; /* no grid, no leaves, no meta section */
  uint32_t M = coord_bits(dtype);
  if (get_u64le(s + 112) != n * dims * M || get_u64le(s + 120) != 0) return BBXO_ECORRUPT;
  if (size < HEADER_BYTES + words_bytes(n * dims * M)) return BBXO_ECORRUPT;
  if (pos_cap_bytes < n * dims * (M / 8)) return BBXO_ENOSPC;
  const uint8_t* pay = s + HEADER_BYTES;
  uint64_t at = 0;
  for (uint64_t i = 0; i < n; i++)
    for (uint32_t d = 0; d < dims; d++, at += M) {
      uint64_t raw = get_bits(pay, at, M);
      uint64_t kk = (layout == 0) ? i * dims + d : (uint64_t)d * n + i;
      if (dtype == 0) {
        uint32_t u32 = (uint32_t)raw;
        memcpy((float*)pos + kk, &u32, 4);
      } else {
        memcpy((double*)pos + kk, &raw, 8);
      }
    }
  return BBXO_OK;
}

/* ------------------------------------------------------------------ sequence export */

/* The sequence layout of Sec. 4.2 (figure fig:sequences), written from a
 * stream whose references are stored as their original coordinates
 * (ref_mode 1).  One sequence per leaf, in stored order: the centre (the
 * reference's coordinates, M bits per axis), the widths m_d (mbits each),
 * the codes of the other members (per member, per axis, m_d bits: the
 * leaf's payload segment) and a 32-bit end mark (all ones).  Bit i is bit
 * i mod 8 of byte i/8; the whole is zero-padded to 8 bytes.  Its length in
 * bits is the storage-cost model of Sec. 4.2 with one sequence per leaf. */
#define END_MARK 0xffffffffu

int bbxo_export_sequences(const uint8_t* s, uint64_t size, uint8_t* out, uint64_t out_cap,
                          uint64_t* out_size) {
  if (!s || size < HEADER_BYTES) return BBXO_ECORRUPT;
  if (get_u32le(s) != MAGIC || get_u16le(s + 4) != 1) return BBXO_ECORRUPT;
  int dtype = s[6];
  uint32_t dims = s[7], r = get_u32le(s + 16), mbits = s[23];
  uint64_t n = get_u64le(s + 8);
  if (dtype > 1 || (dims != 2 && dims != 3) || s[22] > 1 || r == 0) return BBXO_ECORRUPT;
  if (s[22] != 1) return BBXO_EINVAL; /* the centre must be stored losslessly */
  uint32_t M = coord_bits(dtype);
  uint64_t nl = get_u64le(s + 96), meta_bits = get_u64le(s + 104), payload_bits = get_u64le(s + 112);
  if (nl != bbxo_leaf_count(n, r) || meta_bits != nl * (uint64_t)(dims * (mbits + M)))
    return BBXO_ECORRUPT;
  uint64_t mb = words_bytes(meta_bits), pb = words_bytes(payload_bits);
  if (size < HEADER_BYTES + mb + pb) return BBXO_ECORRUPT;
  uint64_t total = nl * (uint64_t)(dims * (M + mbits) + 32) + payload_bits;
  if (out_size) *out_size = words_bytes(total);
  if (words_bytes(total) > out_cap) return BBXO_ENOSPC;
  if (total) memset(out, 0, (size_t)words_bytes(total));
  if (n == 0) return BBXO_OK;
  uint32_t* sizes = (uint32_t*)malloc((size_t)nl * sizeof(uint32_t));
  if (!sizes) return BBXO_ENOMEM;
  uint64_t k = 0;
  size_leaves(n, r, sizes, &k, nl);
  const uint8_t* meta = s + HEADER_BYTES;
  const uint8_t* pay = meta + mb;
  uint64_t mpos = 0, ppos = 0, opos = 0;
  int st = BBXO_OK;
  for (uint64_t i = 0; i < nl; i++) {
    uint32_t m[3] = {0, 0, 0}, sm = 0;
    for (uint32_t d = 0; d < dims; d++) m[d] = (uint32_t)get_bits(meta, mpos + d * mbits, mbits), sm += m[d];
    for (uint32_t d = 0; d < dims; d++) /* centre first */
      put_bits(out, opos, get_bits(meta, mpos + dims * mbits + d * M, M), M), opos += M;
    for (uint32_t d = 0; d < dims; d++) put_bits(out, opos, m[d], mbits), opos += mbits;
    mpos += dims * (mbits + M);
    uint64_t len = (uint64_t)(sizes[i] - 1) * sm;
    if (ppos + len > payload_bits) {
      st = BBXO_ECORRUPT;
      break;
    }
    for (uint64_t b = 0; b < len; b += 64) {
      uint32_t c = len - b < 64 ? (uint32_t)(len - b) : 64u;
      put_bits(out, opos + b, get_bits(pay, ppos + b, c), c);
    }
    ppos += len;
    opos += len;
    put_bits(out, opos, END_MARK, 32), opos += 32;
  }
  if (st == BBXO_OK && (ppos != payload_bits || opos != total)) st = BBXO_ECORRUPT;
  free(sizes);
  return st;
}

/* ------------------------------------------------------------------ reordered export */

/* The two reorderings of Sec. 4.2 before entropy coding, applied to the
 * sequence layout: sequences in ascending sum_d m_d (ties in stored order),
 * and inside each sequence the members in ascending R-index (ties in stored
 * order).  Two steps, each exported on its own so that it can be checked
 * against the paper's example:
 *   bbxo_axis_order_by_entropy: the axes in ascending entropy of the
 *     empirical distribution of their widths m_d over all sequences (the
 *     paper's example: m_x uniform on 2..4, m_y uniform on 2..9 and m_z
 *     single-peaked on 2..9 give the order (x, z, y));
 *   bbxo_r_index: a member's codes concatenated in that axis order, the
 *     first axis the most significant part (the paper's example: codes
 *     (01, 100111, 01010) in the order (x, z, y) give 0101010100111). */
typedef struct {
  uint64_t key; /* sum of widths */
  uint64_t idx;
} seqkey_t;
static int cmp_seq(const void* a, const void* b) {
  const seqkey_t *x = (const seqkey_t*)a, *y = (const seqkey_t*)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  return x->idx < y->idx ? -1 : (x->idx > y->idx);
}

/* Entropy -sum p log2 p of each axis' widths, compared exactly as counts:
 * with N sequences in common, H_a < H_b iff sum c log2 c over a's counts
 * exceeds the same sum for b.  Ties keep the lower axis first. */
void bbxo_axis_order_by_entropy(const uint32_t* widths, uint64_t nseq, uint32_t dims,
                                uint32_t* order) {
  uint64_t cnt[3][65];
  memset(cnt, 0, sizeof(cnt));
  for (uint64_t i = 0; i < nseq; i++)
    for (uint32_t d = 0; d < dims; d++) cnt[d][widths[(uint64_t)dims * i + d] & 63]++;
  double sclog[3] = {0, 0, 0};
  for (uint32_t d = 0; d < dims; d++)
    for (int w = 0; w < 65; w++)
      if (cnt[d][w]) sclog[d] += (double)cnt[d][w] * log2((double)cnt[d][w]);
  uint32_t ord[3] = {0, 1, 2};
  /* insertion sort on ascending entropy (descending sum c log2 c), stable */
  for (uint32_t b = 1; b < dims; b++)
    for (uint32_t a = b; a > 0; a--) {
#if MUT(19)
      int before = sclog[ord[a]] < sclog[ord[a - 1]]; /* descending entropy */
#else
      int before = sclog[ord[a]] > sclog[ord[a - 1]];
#endif
      if (!before) break;
      uint32_t t = ord[a];
      ord[a] = ord[a - 1];
      ord[a - 1] = t;
    }
  for (uint32_t d = 0; d < dims; d++) order[d] = ord[d];
}

/* R-index of one member: codes u[d] of m[d] bits concatenated with the axes
 * in the given order, the first axis most significant.  At most 3 * 31 bits:
 * the high 64 bits go to *hi, the low 64 bits are returned. */
uint64_t bbxo_r_index(const uint64_t* u, const uint32_t* m, uint32_t dims, const uint32_t* order,
                      uint64_t* hi) {
  uint64_t h = 0, l = 0;
  for (uint32_t k = 0; k < dims; k++) {
#if MUT(20)
    uint32_t d = order[dims - 1 - k]; /* most significant part last */
#else
    uint32_t d = order[k];
#endif
    uint32_t w = m[d];
    uint64_t v = w ? (u[d] & (w >= 64 ? ~0ull : ((1ull << w) - 1))) : 0;
    /* (h, l) <<= w, then or in v */
    if (w >= 64) {
      h = l;
      l = 0;
    } else if (w > 0) {
      h = (h << w) | (l >> (64 - w));
      l <<= w;
    }
    l |= v;
  }
  if (hi) *hi = h;
  return l;
}

typedef struct {
  uint64_t hi, lo; /* R-index */
  uint64_t u[3];
  uint32_t pos;
} memkey_t;
static int cmp_mem(const void* a, const void* b) {
  const memkey_t *x = (const memkey_t*)a, *y = (const memkey_t*)b;
  if (x->hi != y->hi) return x->hi < y->hi ? -1 : 1;
  if (x->lo != y->lo) return x->lo < y->lo ? -1 : 1;
  return x->pos < y->pos ? -1 : (x->pos > y->pos);
}

int bbxo_export_sequences_reordered(const uint8_t* s, uint64_t size, uint8_t* out,
                                    uint64_t out_cap, uint64_t* out_size, uint32_t* axis_order) {
  uint64_t plain_size = 0;
  int st = bbxo_export_sequences(s, size, NULL, 0, &plain_size);
  if (st != BBXO_ENOSPC && st != BBXO_OK) return st;
  if (out_size) *out_size = plain_size;
  if (plain_size > out_cap) return BBXO_ENOSPC;
  uint8_t* plain = (uint8_t*)calloc((size_t)(plain_size ? plain_size : 8), 1);
  if (!plain) return BBXO_ENOMEM;
  st = bbxo_export_sequences(s, size, plain, plain_size, &plain_size);
  if (st) {
    free(plain);
    return st;
  }
  int dtype = s[6];
  uint32_t dims = s[7], r = get_u32le(s + 16), mbits = s[23], M = coord_bits(dtype);
  uint64_t n = get_u64le(s + 8), nl = get_u64le(s + 96);
  if (plain_size) memset(out, 0, (size_t)plain_size);
  /* widths and offsets of every sequence in the plain layout */
  uint32_t* sizes = (uint32_t*)malloc((size_t)(nl ? nl : 1) * sizeof(uint32_t));
  uint64_t* start = (uint64_t*)malloc((size_t)(nl ? nl : 1) * sizeof(uint64_t));
  uint32_t* wid = (uint32_t*)malloc((size_t)(nl ? nl : 1) * 3 * sizeof(uint32_t));
  seqkey_t* seq = (seqkey_t*)malloc((size_t)(nl ? nl : 1) * sizeof(seqkey_t));
  memkey_t* mem = (memkey_t*)malloc((size_t)(r + 1) * sizeof(memkey_t));
  if (!sizes || !start || !wid || !seq || !mem) {
    free(plain), free(sizes), free(start), free(wid), free(seq), free(mem);
    return BBXO_ENOMEM;
  }
  uint64_t k = 0;
  if (n) size_leaves(n, r, sizes, &k, nl);
  uint64_t pos = 0;
  for (uint64_t i = 0; i < nl; i++) {
    uint32_t sm = 0;
    start[i] = pos;
    for (uint32_t d = 0; d < dims; d++) {
      wid[3 * i + d] = (uint32_t)get_bits(plain, pos + dims * M + d * mbits, mbits);
      sm += wid[3 * i + d];
    }
    seq[i].key = sm;
    seq[i].idx = i;
    pos += dims * (M + mbits) + (uint64_t)(sizes[i] - 1) * sm + 32;
  }
  /* the axis order of the R-index, from every sequence's widths */
  uint32_t* wd = (uint32_t*)malloc((size_t)(nl ? nl : 1) * dims * sizeof(uint32_t));
  if (!wd) {
    free(plain), free(sizes), free(start), free(wid), free(seq), free(mem);
    return BBXO_ENOMEM;
  }
  for (uint64_t i = 0; i < nl; i++)
    for (uint32_t d = 0; d < dims; d++) wd[(uint64_t)dims * i + d] = wid[3 * i + d];
  uint32_t ord[3] = {0, 1, 2};
  bbxo_axis_order_by_entropy(wd, nl, dims, ord);
  free(wd);
  if (axis_order)
    for (uint32_t d = 0; d < dims; d++) axis_order[d] = ord[d];
  qsort(seq, (size_t)nl, sizeof(seqkey_t), cmp_seq);
  uint64_t opos = 0;
  for (uint64_t q = 0; q < nl; q++) {
    uint64_t i = seq[q].idx, ip = start[i];
    const uint32_t* m = wid + 3 * i;
    uint32_t hdr = dims * (M + mbits), sm = (uint32_t)seq[q].key;
    for (uint32_t b = 0; b < hdr; b += 32) {
      uint32_t c = hdr - b < 32 ? hdr - b : 32;
      put_bits(out, opos + b, get_bits(plain, ip + b, c), c);
    }
    uint64_t cp = ip + hdr, op = opos + hdr;
    uint32_t cntm = sizes[i] - 1;
    for (uint32_t j = 0; j < cntm; j++) {
      mem[j].pos = j;
      uint64_t at = cp + (uint64_t)j * sm;
      for (uint32_t d = 0; d < 3; d++) {
        mem[j].u[d] = 0;
        if (d < dims) {
          mem[j].u[d] = get_bits(plain, at, m[d]);
          at += m[d];
        }
      }
    }
    for (uint32_t j = 0; j < cntm; j++) mem[j].lo = bbxo_r_index(mem[j].u, m, dims, ord, &mem[j].hi);
    qsort(mem, cntm, sizeof(memkey_t), cmp_mem);
    for (uint32_t j = 0; j < cntm; j++)
      for (uint32_t d = 0; d < dims; d++) put_bits(out, op, mem[j].u[d], m[d]), op += m[d];
    put_bits(out, op, END_MARK, 32);
    opos = op + 32;
  }
  free(plain), free(sizes), free(start), free(wid), free(seq), free(mem);
  return BBXO_OK;
}

/* ------------------------------------------------------------------ entropy coding */

/* Huffman coding of a byte sequence (the encoding phase of Sec. 3, which the
 * paper applies to its sequence layout, Sec. 4.2).  Symbols are bytes.  Code
 * lengths come from Huffman's construction: repeatedly the two lightest
 * nodes merge, weights compared first and the node created earlier (leaves
 * first, in symbol order) preferred on ties; a tree deeper than HUF_MAXLEN
 * is rebuilt from the weights halved (rounded up, so none vanishes) until
 * it fits.  Codes are canonical: symbols in (length, symbol) order take
 * consecutive codes, each shifted left when the length grows.  The input is
 * cut into chunks of HUF_CHUNK bytes whose first bit offsets are stored, so
 * chunks decode independently.
 *
 * Stream: [0,4) 'BBXH' | [4,6) version 1 | [6] HUF_MAXLEN | [7] 0 |
 * [8,16) n bytes | [16,20) HUF_CHUNK | [20,24) 0 | [24,32) chunks |
 * [32,40) payload bits | [40,48) 0 | [48,176) code lengths, a nibble per
 * symbol (low nibble: even symbol) | chunk bit offsets (u64 each, from the
 * payload start) | payload: codes in input order, each code's most
 * significant bit first, bit i of the payload = bit i mod 64 of its u64 word
 * i / 64, zero-padded to 8 bytes. */
#define HUF_MAGIC 0x48584242u /* bytes 'B','B','X','H' */
#define HUF_MAXLEN 12u
#define HUF_CHUNK 4096u
#define HUF_HEADER 176u

void bbxo_huffman_lengths(const uint64_t* counts, uint32_t* len) {
  uint64_t w[256];
  for (int s = 0; s < 256; s++) w[s] = counts[s], len[s] = 0;
  for (;;) {
    uint32_t sym[256], k = 0;
    for (uint32_t s = 0; s < 256; s++)
      if (w[s]) sym[k++] = s;
    if (k == 0) return;
    if (k == 1) {
      len[sym[0]] = 1;
      return;
    }
    /* nodes 0..k-1 the leaves (symbol order), k.. the merged ones */
    uint64_t weight[511];
    int parent[511], alive[511];
    for (uint32_t i = 0; i < k; i++) weight[i] = w[sym[i]], parent[i] = -1, alive[i] = 1;
    uint32_t nn = k;
    for (uint32_t m = 0; m + 1 < k; m++) {
      int pick[2] = {-1, -1};
      for (int t = 0; t < 2; t++)
        for (uint32_t i = 0; i < nn; i++) {
          if (!alive[i] || (int)i == pick[0]) continue;
#if MUT(35)
          if (pick[t] < 0 || weight[i] > weight[pick[t]]) pick[t] = (int)i; /* heaviest */
#elif MUT(33)
          if (pick[t] < 0 || weight[i] <= weight[pick[t]]) pick[t] = (int)i; /* later on ties */
#else
          if (pick[t] < 0 || weight[i] < weight[pick[t]]) pick[t] = (int)i;
#endif
        }
      weight[nn] = weight[pick[0]] + weight[pick[1]];
      parent[nn] = -1;
      alive[nn] = 1;
      alive[pick[0]] = alive[pick[1]] = 0;
      parent[pick[0]] = parent[pick[1]] = (int)nn;
      nn++;
    }
    uint32_t deepest = 0, d[256];
    for (uint32_t i = 0; i < k; i++) {
      uint32_t depth = 0;
      for (int p = parent[i]; p >= 0; p = parent[p]) depth++;
      d[i] = depth;
      if (depth > deepest) deepest = depth;
    }
    if (deepest <= HUF_MAXLEN) {
      for (uint32_t i = 0; i < k; i++) len[sym[i]] = d[i];
      return;
    }
    for (int s = 0; s < 256; s++)
      if (w[s]) w[s] = (w[s] + 1) / 2;
  }
}

/* Canonical codes of the lengths. */
static void huf_codes(const uint32_t* len, uint32_t* code) {
  uint32_t c = 0, prev = 0;
  int first = 1;
  for (uint32_t L = 1; L <= HUF_MAXLEN; L++)
#if MUT(34)
    for (int s = 255; s >= 0; s--) {
#else
    for (int s = 0; s < 256; s++) {
#endif
      if (len[s] != L) continue;
      if (!first) c = (c + 1) << (L - prev);
      first = 0;
      code[s] = c;
      prev = L;
    }
}

static void put_code(uint8_t* sec, uint64_t pos, uint32_t code, uint32_t L) {
  for (uint32_t b = 0; b < L; b++) {
#if MUT(37)
    uint32_t bit = (code >> b) & 1u; /* least significant bit first */
#else
    uint32_t bit = (code >> (L - 1 - b)) & 1u;
#endif
    if (bit) sec[(pos + b) >> 3] |= (uint8_t)(1u << ((pos + b) & 7u));
  }
}

uint64_t bbxo_huffman_bound(uint64_t n) {
  return HUF_HEADER + 8 * ((n + HUF_CHUNK - 1) / HUF_CHUNK) + words_bytes(n * HUF_MAXLEN);
}

int bbxo_huffman_encode(const uint8_t* in, uint64_t n, uint8_t* out, uint64_t out_cap,
                        uint64_t* out_size) {
  uint64_t cnt[256];
  uint32_t len[256], code[256];
  memset(cnt, 0, sizeof(cnt));
  for (uint64_t i = 0; i < n; i++) cnt[in[i]]++;
  bbxo_huffman_lengths(cnt, len);
  memset(code, 0, sizeof(code));
  huf_codes(len, code);
  uint64_t bits = 0;
  for (int s = 0; s < 256; s++) bits += cnt[s] * len[s];
  const uint64_t chunks = (n + HUF_CHUNK - 1) / HUF_CHUNK;
  const uint64_t total = HUF_HEADER + 8 * chunks + words_bytes(bits);
  if (out_size) *out_size = total;
  if (total > out_cap) return BBXO_ENOSPC;
  memset(out, 0, (size_t)total);
  put_u32le(out, HUF_MAGIC);
  put_u16le(out + 4, 1);
  out[6] = (uint8_t)HUF_MAXLEN;
  put_u64le(out + 8, n);
  put_u32le(out + 16, HUF_CHUNK);
  put_u64le(out + 24, chunks);
  put_u64le(out + 32, bits);
  for (int s = 0; s < 256; s++) out[48 + s / 2] |= (uint8_t)(len[s] << ((s & 1) ? 4 : 0));
  uint8_t* offs = out + HUF_HEADER;
  uint8_t* pay = offs + 8 * chunks;
  uint64_t pos = 0;
  for (uint64_t i = 0; i < n; i++) {
    if (i % HUF_CHUNK == 0)
#if MUT(36)
      put_u64le(offs + 8 * (i / HUF_CHUNK), pos + (i ? 1 : 0));
#else
      put_u64le(offs + 8 * (i / HUF_CHUNK), pos);
#endif
    put_code(pay, pos, code[in[i]], len[in[i]]);
    pos += len[in[i]];
  }
  return BBXO_OK;
}

int bbxo_huffman_decode(const uint8_t* s, uint64_t size, uint8_t* out, uint64_t out_cap,
                        uint64_t* out_n) {
  if (!s || size < HUF_HEADER || get_u32le(s) != HUF_MAGIC || get_u16le(s + 4) != 1 ||
      s[6] != HUF_MAXLEN || s[7] != 0 || get_u32le(s + 16) != HUF_CHUNK || get_u32le(s + 20) != 0 ||
      get_u64le(s + 40) != 0)
    return BBXO_ECORRUPT;
  const uint64_t n = get_u64le(s + 8), chunks = get_u64le(s + 24), bits = get_u64le(s + 32);
  if (chunks != (n + HUF_CHUNK - 1) / HUF_CHUNK || bits > n * HUF_MAXLEN) return BBXO_ECORRUPT;
  if (size < HUF_HEADER + 8 * chunks + words_bytes(bits)) return BBXO_ECORRUPT;
  if (out_n) *out_n = n;
  if (n > out_cap) return BBXO_ENOSPC;
  uint32_t len[256], code[256];
  uint64_t kraft = 0; /* in units of 2^-HUF_MAXLEN */
  uint32_t used = 0;
  for (int t = 0; t < 256; t++) {
    len[t] = (s[48 + t / 2] >> ((t & 1) ? 4 : 0)) & 15u;
    if (len[t] > HUF_MAXLEN) return BBXO_ECORRUPT;
    if (len[t]) kraft += 1ull << (HUF_MAXLEN - len[t]), used++;
  }
  if (n > 0 && (used == 0 || kraft > (1ull << HUF_MAXLEN))) return BBXO_ECORRUPT;
  memset(code, 0, sizeof(code));
  huf_codes(len, code);
  const uint8_t* offs = s + HUF_HEADER;
  const uint8_t* pay = offs + 8 * chunks;
  for (uint64_t c = 0; c < chunks; c++) {
    uint64_t pos = get_u64le(offs + 8 * c);
    const uint64_t end = c + 1 < chunks ? get_u64le(offs + 8 * (c + 1)) : bits;
    if (pos > end || end > bits) return BBXO_ECORRUPT;
    const uint64_t i0 = c * HUF_CHUNK, i1 = i0 + HUF_CHUNK < n ? i0 + HUF_CHUNK : n;
    for (uint64_t i = i0; i < i1; i++) {
      /* read bits until they spell a code of the table */
      uint32_t v = 0, L = 0, sym = 256;
      while (sym == 256) {
        if (L == HUF_MAXLEN || pos >= end) return BBXO_ECORRUPT;
        v = (v << 1) | (uint32_t)((pay[pos >> 3] >> (pos & 7u)) & 1u);
        pos++, L++;
        for (int t = 0; t < 256 && sym == 256; t++)
          if (len[t] == L && code[t] == v) sym = (uint32_t)t;
      }
      out[i] = (uint8_t)sym;
    }
    if (pos != end) return BBXO_ECORRUPT;
  }
  return BBXO_OK;
}

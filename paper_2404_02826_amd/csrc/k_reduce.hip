// k_reduce.hip -- the bit box reduction of Sec. 4.1 (the while loop of
// Alg. 1) after the partition and leaf bit boxes, and its stream (format
// version 2: one meta record per sequence with a 32-bit particle count).
//
// The reduction repeatedly takes the remaining box with the smallest key
// (sum of widths, or with reduce = 2 the sum of Eq. 3 box lengths), ties to
// the first leaf in depth-first order.  Its sequence is its reference, its
// other remaining members in ascending index, then the "common" particles:
// the remaining members of every other remaining box whose bit box meets
// the popped one and that lie inside the popped box, box by box in leaf
// order, each box's in ascending index.  A box that lost particles gets a
// new bit box from what it keeps (AABB, member nearest the AABB centre,
// Eq. 2); an empty one vanishes.  In code space a bit box of reference
// codes c and widths m holds the codes q with |q_d - c_d| <= 2^(m_d-1) - 1
// (nothing but c_d when m_d = 0), the offsets its widths can encode.
//
// Every pop depends on the state the previous one left, so one workgroup
// runs a set's loop; the work inside a pop (the smallest key over all boxes,
// which boxes meet the popped one, which particles they lose, the new bit
// boxes) is spread over the workgroup, and the sets of a batch run in
// parallel, one workgroup each.
//
//   k_red_prep      per leaf: its members in ascending index (the leaf
//                   stage writes them reference first), their codes and
//                   source indices side by side, the leaf's box and key
//   k_reduce        the loop, one workgroup per set
//   k_red_meta      meta records (widths, centre codes, count)
//   k_red_payload   payload words, gathered (one thread per word)
//   k_red_perm      source index of every output slot
// Decoding (version 2): k_dec_meta2 per sequence, scans of the slot counts
// and payload bits, k_unpack2 one thread per output slot.
#include "bbx_internal.h"

namespace bbx {

typedef unsigned __int128 u128;

constexpr uint64_t kDead = ~0ull;  // key of a popped or empty box

__device__ inline uint32_t red_reach(uint32_t m) { return m ? (1u << (m - 1)) - 1u : 0u; }

// The reduction state of a set inside the batch workspace.
struct RedSet {
  uint4* tq;          // [n] codes (x, y, z) and source index, leaves' members in ascending index
  uint8_t* taken;     // [n] 1 once a particle is in a sequence
  uint32_t* slot_pos; // [n] tq position of each output slot
  uint64_t* key;      // [n_leaves] key << 31 | leaf, or kDead
  uint4* ctr;         // [n_leaves] the box: its reference's codes (x, y, z) and packed widths
  uint32_t* ref;      // [n_leaves] tq position of the box's reference
  uint32_t* hits;     // [n_leaves] boxes meeting the popped one
  uint4* seq;         // [n_leaves] centre position, packed widths, count, first slot
};

__device__ inline RedSet red_set(const SetDesc& S, const Ws& w) {
  RedSet r;
  r.tq = w.red_tq + S.idx_off;
  r.taken = w.red_taken + S.idx_off;
  r.slot_pos = w.red_slot + S.idx_off;
  r.key = w.red_key + S.leaf_off;
  r.ctr = w.red_ctr + S.leaf_off;
  r.ref = w.red_ref + S.leaf_off;
  r.hits = w.red_hits + S.leaf_off;
  r.seq = w.red_seq + S.leaf_off;
  return r;
}

// ---------------------------------------------------------------- preparation

template <typename KT>
__device__ void red_prep_leaf(const SetDesc& S, const RedSet& R, const KT* keys, const uint32_t* src,
                              const LeafRec& rec, uint32_t leaf) {
  const uint32_t st = rec.start, sz = rec.size;
  const uint32_t sref = src[st];
  // the reference's place among the others (they are in ascending index)
  uint32_t rr = 0;
  for (uint32_t k = 1; k < sz; ++k) rr += src[st + k] < sref ? 1u : 0u;
  for (uint32_t k = 0; k < sz; ++k) {
    const uint32_t slot = st + k, sk = src[slot];
    const uint32_t tp = k == 0 ? st + rr : st + (k - 1) + (sk > sref ? 1u : 0u);
    uint4 v;
    v.x = keys[slot];
    v.y = S.dims > 1 ? (uint32_t)keys[S.kst + slot] : 0u;
    v.z = S.dims > 2 ? (uint32_t)keys[2 * S.kst + slot] : 0u;
    v.w = sk;
    R.tq[tp] = v;
    R.taken[tp] = 0;
  }
  R.ref[leaf] = st + rr;
  R.ctr[leaf] = make_uint4(rec.qref[0], rec.qref[1], rec.qref[2], rec.m);
  R.key[leaf] = red_key(rec.m, S.dims, S.reduce, leaf);
}

__global__ void __launch_bounds__(kBlock) k_red_prep(uint32_t nsets, const uint64_t* pre, Ws w) {
  const uint32_t s = find_set(pre, nsets, blockIdx.x);
  const SetDesc& S = w.sets[s];
  const DevParams* P = w.params + s;
  if (P->status != BBX_OK || !S.reduce) return;
  const uint64_t leaf = (blockIdx.x - pre[s]) * kBlock + threadIdx.x;
  if (leaf >= S.n_leaves) return;
  const RedSet R = red_set(S, w);
  const uint8_t* keys = (S.final_buf ? w.keys[1] : w.keys[0]) + S.key_off;
  const LeafRec rec = w.leaves[S.leaf_off + leaf];
  if (P->key16)
    red_prep_leaf(S, R, (const uint16_t*)keys, S.perm, rec, (uint32_t)leaf);
  else
    red_prep_leaf(S, R, (const uint32_t*)keys, S.perm, rec, (uint32_t)leaf);
}

// ---------------------------------------------------------------- the loop

__device__ inline uint64_t wave_min_u64(uint64_t x) {
  for (int o = 32; o > 0; o >>= 1) {
    const uint64_t y = __shfl_xor(x, o);
    x = y < x ? y : x;
  }
  return x;
}

// A leaf's members: positions [st, st + sz) of the set's tq array.
struct RedLeaf {
  uint32_t st, sz;
};

__device__ inline bool red_inside(const uint4 q, const uint32_t c[3], const uint32_t R[3],
                                  uint32_t dims) {
  bool in = true;
  const uint32_t v[3] = {q.x, q.y, q.z};
  for (uint32_t d = 0; d < dims; ++d) {
    const uint32_t o = v[d] > c[d] ? v[d] - c[d] : c[d] - v[d];
    in = in && o <= R[d];
  }
  return in;
}

// Whether box b (reference codes and packed widths) meets the popped box:
// the code intervals overlap on every axis.
__device__ inline bool red_meet(const uint4 b, const uint32_t c[3], const uint32_t R[3],
                                uint32_t dims) {
  bool hit = true;
  const uint32_t o[3] = {b.x, b.y, b.z};
  for (uint32_t d = 0; d < dims; ++d) {
    const uint64_t gap = o[d] > c[d] ? o[d] - c[d] : c[d] - o[d];
    hit = hit && gap <= (uint64_t)R[d] + red_reach(red_m(b.w, d));
  }
  return hit;
}

// Bit box of the members of [st, st + sz) that stay: not taken before this
// pop and not inside the popped box (c, Rr).  AABB, the member nearest the
// AABB centre (squared distance in doubled code space, first position on
// ties), Eq. 2.  One wavefront; reads the taken flags only (the caller marks
// the popped box's catch afterwards).
__device__ inline void red_refit(const RedSet& R, uint32_t st, uint32_t sz, uint32_t dims,
                                 const uint32_t c[3], const uint32_t Rr[3], uint32_t* ref_out,
                                 uint4* box_out) {
  const uint32_t lane = threadIdx.x & 63;
  uint32_t mn[3] = {~0u, ~0u, ~0u}, mx[3] = {0, 0, 0};
  for (uint32_t k = lane; k < sz; k += 64) {
    if (R.taken[st + k]) continue;
    const uint4 q = R.tq[st + k];
    if (red_inside(q, c, Rr, dims)) continue;
    const uint32_t v[3] = {q.x, q.y, q.z};
    for (uint32_t d = 0; d < 3; ++d) mn[d] = umin32(mn[d], v[d]), mx[d] = umax32(mx[d], v[d]);
  }
  for (uint32_t d = 0; d < 3; ++d) mn[d] = wave_min_dpp(mn[d]), mx[d] = wave_max_dpp(mx[d]);
  uint64_t bd = kDead;
  uint32_t bk = ~0u;
  for (uint32_t k = lane; k < sz; k += 64) {
    if (R.taken[st + k]) continue;
    const uint4 q = R.tq[st + k];
    if (red_inside(q, c, Rr, dims)) continue;
    const uint32_t v[3] = {q.x, q.y, q.z};
    uint64_t dist = 0;
    for (uint32_t d = 0; d < dims; ++d) {
      const int64_t t = 2 * (int64_t)v[d] - (int64_t)mn[d] - (int64_t)mx[d];
      dist += (uint64_t)(t * t);
    }
    if (dist < bd) bd = dist, bk = k;  // k ascends within a lane: the first on ties
  }
  for (int o = 32; o > 0; o >>= 1) {
    const uint64_t od = __shfl_xor(bd, o);
    const uint32_t ok = (uint32_t)__shfl_xor((int)bk, o);
    if (od < bd || (od == bd && ok < bk)) bd = od, bk = ok;
  }
  const uint4 q = R.tq[st + bk];
  const uint32_t v[3] = {q.x, q.y, q.z};
  uint32_t mp = 0;
  for (uint32_t d = 0; d < dims; ++d) {
    const uint32_t D = umax32(v[d] - mn[d], mx[d] - v[d]);
    mp |= red_width(D) << (8 * d);
  }
  *ref_out = st + bk;
  *box_out = make_uint4(v[0], v[1], v[2], mp);
}

// threads of the reduction loop: the pops' box scans and their catch are
// spread over 16 wavefronts
constexpr uint32_t kRedBlock = 1024;

// Block-wide exclusive scan of one count per thread; *total gets the sum.
__device__ inline uint32_t red_exscan(uint32_t v, uint32_t* wsum, uint32_t* total) {
  const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint32_t incl = wave_incl(v);
  if (lane == 63) wsum[wv] = incl;
  __syncthreads();
  uint32_t off = 0, tot = 0;
  for (uint32_t k = 0; k < kRedBlock / 64; ++k) {
    off += k < wv ? wsum[k] : 0u;
    tot += wsum[k];
  }
  *total = tot;
  return off + incl - v;
}

// The loop of one set.  LDS: the boxes' keys and records live in on-chip
// memory for the whole loop (sets of at most kRedLdsBoxes leaves); else in
// the workspace.  Each thread owns a contiguous range of boxes for the two
// scans of every pop (smallest key; boxes that meet the popped one).
template <bool LDS>
__global__ void __launch_bounds__(kRedBlock) k_reduce(uint32_t nsets, const uint64_t* pre, Ws w) {
  extern __shared__ __align__(16) uint8_t red_dyn[];
  const uint32_t s = find_set(pre, nsets, blockIdx.x);
  const SetDesc& S = w.sets[s];
  DevParams* P = w.params + s;
  if (P->status != BBX_OK || !S.reduce || S.n == 0) return;
  // a split-rule set's leaf count is found on the device
  const uint64_t NL = S.split ? P->nleaves : S.n_leaves;
  if ((NL <= kRedLdsBoxes) != LDS) return;
  const RedSet R = red_set(S, w);
  const LeafRec* leaves = w.leaves + S.leaf_off;
  const uint32_t B = (uint32_t)NL, dims = S.dims;
  const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  constexpr uint32_t W = kRedBlock / 64;
  uint64_t* K = LDS ? (uint64_t*)red_dyn : R.key;
  uint4* C = LDS ? (uint4*)(red_dyn + 8 * (size_t)kRedLdsBoxes) : R.ctr;
  __shared__ uint64_t s_min[W];
  __shared__ uint32_t s_cnt[W], s_wsum[W];
  __shared__ uint32_t s_slot, s_nseq, s_first;
  if (LDS)
    for (uint32_t b = threadIdx.x; b < B; b += kRedBlock) K[b] = R.key[b], C[b] = R.ctr[b];
  if (threadIdx.x == 0) s_slot = 0, s_nseq = 0;
  __syncthreads();
  const uint32_t per = (B + kRedBlock - 1) / kRedBlock;
  const uint32_t b_lo = umin32(threadIdx.x * per, B), b_hi = umin32(b_lo + per, B);
  for (;;) {
    // ---- the remaining box with the smallest (key, leaf)
    uint64_t best = kDead;
    for (uint32_t b = b_lo; b < b_hi; ++b) {
      const uint64_t k = K[b];
      best = k < best ? k : best;
    }
    best = wave_min_u64(best);
    if (lane == 0) s_min[wv] = best;
    __syncthreads();
    best = s_min[0];
    for (uint32_t k = 1; k < W; ++k) best = s_min[k] < best ? s_min[k] : best;
    if (best == kDead) break;  // uniform: every box popped or empty
    const uint32_t cur = (uint32_t)(best & 0x7fffffffu);
    const uint4 cb = C[cur];
    const uint32_t c[3] = {cb.x, cb.y, cb.z};
    const uint32_t Rr[3] = {red_reach(red_m(cb.w, 0)), red_reach(red_m(cb.w, 1)),
                            red_reach(red_m(cb.w, 2))};
    const uint32_t first = s_slot;
    // ---- its centre, then its other remaining members in ascending index
    // (wavefront 0, while the others start the scan below; it skips cur)
    if (wv == 0) {
      const uint32_t cref = R.ref[cur];
      const RedLeaf L = {leaves[cur].start, leaves[cur].size};
      uint32_t at = first + 1;
      for (uint32_t k0 = 0; k0 < L.sz; k0 += 64) {
        const uint32_t k = k0 + lane;
        const bool mine = k < L.sz && L.st + k != cref && !R.taken[L.st + k];
        const uint64_t bm = __ballot(mine);
        if (mine && at + lanes_below(bm) < S.n) {
          R.slot_pos[at + lanes_below(bm)] = L.st + k;
          R.taken[L.st + k] = 1;
        }
        at += (uint32_t)__popcll(bm);
      }
      if (lane == 0) {
        if (first < S.n) R.slot_pos[first] = cref;
        R.taken[cref] = 1;
        s_first = at;
      }
    }
    // ---- every other remaining box that meets the popped one, in leaf order
    uint32_t nhit = 0;
    for (uint32_t b = b_lo; b < b_hi; ++b)
      nhit += (b != cur && K[b] != kDead && red_meet(C[b], c, Rr, dims)) ? 1u : 0u;
    uint32_t nh;
    uint32_t at_h = red_exscan(nhit, s_wsum, &nh);
    for (uint32_t b = b_lo; b < b_hi && nhit; ++b)
      if (b != cur && K[b] != kDead && red_meet(C[b], c, Rr, dims)) R.hits[at_h++] = b;
    __syncthreads();
    if (threadIdx.x == 0) K[cur] = kDead;
    // ---- their common particles, W boxes at a time (one wavefront each)
    for (uint32_t h0 = 0; h0 < nh; h0 += W) {
      const uint32_t h = h0 + wv;
      uint32_t b = 0;
      RedLeaf L = {0, 0};
      uint32_t cnt = 0, keep = 0;
      if (h < nh) {
        b = R.hits[h];
        L = {leaves[b].start, leaves[b].size};
        for (uint32_t k0 = 0; k0 < L.sz; k0 += 64) {
          const uint32_t k = k0 + lane;
          bool in = false, alive = false;
          if (k < L.sz && !R.taken[L.st + k]) {
            alive = true;
            in = red_inside(R.tq[L.st + k], c, Rr, dims);
          }
          cnt += (uint32_t)__popcll(__ballot(in));
          keep += (uint32_t)__popcll(__ballot(alive && !in));
        }
      }
      if (lane == 0) s_cnt[wv] = cnt;
      __syncthreads();
      uint32_t at = s_first;
      for (uint32_t k = 0; k < wv; ++k) at += s_cnt[k];
      if (h < nh && cnt > 0) {
        // output slots of the catch, and the box rebuilt from what stays;
        // the taken flags are read by both and set afterwards
        for (uint32_t k0 = 0; k0 < L.sz; k0 += 64) {
          const uint32_t k = k0 + lane;
          const bool in = k < L.sz && !R.taken[L.st + k] && red_inside(R.tq[L.st + k], c, Rr, dims);
          const uint64_t bm = __ballot(in);
          if (in && at + lanes_below(bm) < S.n) R.slot_pos[at + lanes_below(bm)] = L.st + k;
          at += (uint32_t)__popcll(bm);
        }
        uint32_t ref = 0;
        uint4 nb = make_uint4(0, 0, 0, 0);
        if (keep > 0) red_refit(R, L.st, L.sz, dims, c, Rr, &ref, &nb);
        // every lane's reads of this box's flags are done (wavefront order)
        __builtin_amdgcn_wave_barrier();
        for (uint32_t k0 = 0; k0 < L.sz; k0 += 64) {
          const uint32_t k = k0 + lane;
          if (k < L.sz && !R.taken[L.st + k] && red_inside(R.tq[L.st + k], c, Rr, dims))
            R.taken[L.st + k] = 1;
        }
        if (lane == 0) {
          if (keep == 0) {
            K[b] = kDead;  // empty: vanishes
          } else {
            R.ref[b] = ref;
            C[b] = nb;
            K[b] = red_key(nb.w, dims, S.reduce, b);
          }
        }
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (uint32_t k = 0; k < W; ++k) t += s_cnt[k];
        s_first += t;
      }
      __syncthreads();
    }
    // ---- the sequence record
    if (threadIdx.x == 0) {
      R.seq[s_nseq] = make_uint4(R.ref[cur], cb.w, s_first - first - 1, first);
      s_nseq += 1;
      s_slot = s_first;
    }
    __syncthreads();
  }
  const uint32_t nseq = s_nseq;
  if (threadIdx.x == 0) {
    P->nseq = nseq;
    // every particle placed exactly once (slot writes past n were dropped)
    if (s_slot != S.n) check_failed(P, kChkReduce);
  }
  // payload bits per sequence (zero past the last), for the offset scan
  uint64_t* bits = w.leaf_bits + S.leaf_off;
  for (uint32_t i = threadIdx.x; i < B; i += kRedBlock) {
    uint64_t v = 0;
    if (i < nseq) {
      const uint4 q = R.seq[i];
      v = (uint64_t)q.z * (red_m(q.y, 0) + red_m(q.y, 1) + red_m(q.y, 2));
    }
    bits[i] = v;
  }
}

// ---------------------------------------------------------------- packing

__device__ inline void red_or(uint64_t& word, uint64_t w0, u128 val, uint64_t at, uint32_t len) {
  if (len == 0) return;
  const int64_t rel = (int64_t)(at - w0);
  if (rel >= 64 || rel + (int64_t)len <= 0) return;
  if (len < 128) val &= (((u128)1) << len) - 1;
  if (rel >= 0)
    word |= (uint64_t)(val << rel);
  else
    word |= (uint64_t)(val >> (-rel));
}

__global__ void __launch_bounds__(kBlock) k_red_meta(uint32_t nsets, const uint64_t* pre, Ws w) {
  const uint32_t s = find_set(pre, nsets, blockIdx.x);
  const SetDesc& S = w.sets[s];
  const DevParams* P = w.params + s;
  if (P->status != BBX_OK || !seq_stream(S)) return;
  const RedSet R = red_set(S, w);
  const uint64_t lb = blockIdx.x - pre[s], nblk = pre[s + 1] - pre[s];
  const uint32_t dims = S.dims, mbits = S.mbits;
  uint32_t sumG = 0;
  for (uint32_t d = 0; d < dims; ++d) sumG += P->G[d];
  const uint32_t Sb = dims * mbits + sumG + 32;
  const uint64_t nseq = P->nseq, nwords = (P->meta_bits + 63) / 64;
  uint64_t* meta = (uint64_t*)(S.out + kHeaderBytes);
  for (uint64_t wd = lb * kBlock + threadIdx.x; wd < nwords; wd += nblk * kBlock) {
    const uint64_t b0 = wd * 64;
    const uint64_t i0 = b0 / Sb;
    uint64_t i1 = (b0 + 63) / Sb;
    if (i1 >= nseq) i1 = nseq - 1;
    uint64_t word = 0;
    for (uint64_t i = i0; i <= i1; ++i) {
      const uint4 q = R.seq[i];
      const uint4 cq = R.tq[q.x];
      const uint32_t cv[3] = {cq.x, cq.y, cq.z};
      u128 v = 0;
      uint32_t at = 0;
      for (uint32_t d = 0; d < dims; ++d) v |= (u128)red_m(q.y, d) << at, at += mbits;
      for (uint32_t d = 0; d < dims; ++d) v |= (u128)cv[d] << at, at += P->G[d];
      red_or(word, b0, v, i * Sb, at);
      red_or(word, b0, q.z, i * Sb + at, 32);
    }
    meta[wd] = word;
  }
}

// largest i < count with off[i] - base <= b (offsets non-decreasing)
__device__ inline uint64_t red_search(const uint64_t* off, uint64_t base, uint64_t count, uint64_t b) {
  uint64_t lo = 0, hi = count - 1;
  while (lo < hi) {
    const uint64_t mid = lo + (hi - lo + 1) / 2;
    if (off[mid] - base <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

__global__ void __launch_bounds__(kBlock) k_red_payload(uint32_t nsets, const uint64_t* pre, Ws w) {
  const uint32_t s = find_set(pre, nsets, blockIdx.x);
  const SetDesc& S = w.sets[s];
  const DevParams* P = w.params + s;
  if (P->status != BBX_OK || !seq_stream(S) || P->payload_bits == 0) return;
  const RedSet R = red_set(S, w);
  const uint64_t lb = blockIdx.x - pre[s], nblk = pre[s + 1] - pre[s];
  const uint64_t nseq = P->nseq, base = P->payload_base;
  const uint64_t* off = w.leaf_bits + S.leaf_off;
  const uint64_t nwords = (P->payload_bits + 63) / 64;
  const uint32_t dims = S.dims;
  uint64_t* pay = (uint64_t*)(S.out + kHeaderBytes + ((P->meta_bits + 63) / 64) * 8);
  for (uint64_t wd = lb * kBlock + threadIdx.x; wd < nwords; wd += nblk * kBlock) {
    const uint64_t b0 = wd * 64;
    uint64_t word = 0;
    for (uint64_t i = red_search(off, base, nseq, b0); i < nseq; ++i) {
      const uint64_t a = off[i] - base;
      if (a >= b0 + 64) break;
      const uint4 q = R.seq[i];
      const uint32_t m[3] = {red_m(q.y, 0), red_m(q.y, 1), red_m(q.y, 2)};
      const uint32_t sm = m[0] + m[1] + m[2];
      if (sm == 0 || q.z == 0) continue;
      const uint4 cq = R.tq[q.x];
      const uint32_t cv[3] = {cq.x, cq.y, cq.z};
      uint64_t j = b0 > a ? (b0 - a) / sm : 0;
      for (; j < q.z; ++j) {
        const uint64_t at = a + j * sm;
        if (at >= b0 + 64) break;
        const uint4 pq = R.tq[R.slot_pos[q.w + 1 + j]];
        const uint32_t pv[3] = {pq.x, pq.y, pq.z};
        u128 v = 0;
        uint32_t sh = 0;
        for (uint32_t d = 0; d < dims; ++d) {
          if (m[d] == 0) continue;
          const uint32_t u = pv[d] - cv[d] + (1u << (m[d] - 1));
          v |= (u128)u << sh;
          sh += m[d];
        }
        red_or(word, b0, v, at, sm);
      }
    }
    pay[wd] = word;
  }
}

__global__ void __launch_bounds__(kBlock) k_red_perm(uint32_t nsets, const uint64_t* pre, Ws w) {
  const uint32_t s = find_set(pre, nsets, blockIdx.x);
  const SetDesc& S = w.sets[s];
  const DevParams* P = w.params + s;
  if (P->status != BBX_OK || !seq_stream(S) || !S.user_perm) return;
  const RedSet R = red_set(S, w);
  const uint64_t lb = blockIdx.x - pre[s], nblk = pre[s + 1] - pre[s];
  for (uint64_t i = lb * kBlock + threadIdx.x; i < S.n; i += nblk * kBlock)
    S.user_perm[i] = R.tq[R.slot_pos[i]].w;
}

hipError_t launch_reduce(const BatchPlan& bp, const Ws& w, hipStream_t s) {
  if (!bp.reduce) return hipGetLastError();
  // the on-chip variant keeps 24 bytes per box: above the default 64 KB of
  // dynamic LDS, so its limit is raised once (gfx950 has 160 KB per CU)
  static hipError_t lds_set = hipFuncSetAttribute(
      (const void*)k_reduce<true>, hipFuncAttributeMaxDynamicSharedMemorySize, 24 * kRedLdsBoxes);
  if (lds_set != hipSuccess) return lds_set;
  if (bp.g_rp > 0) BBX_LAUNCH("reduce_prep", k_red_prep, bp.g_rp, kBlock, 0, s, bp.nsets, w.pre + bp.o_rp, w);
  if (bp.g_rl > 0) {
    if (bp.red_lds_boxes)
      BBX_LAUNCH("reduce", k_reduce<true>, bp.g_rl, kRedBlock, (size_t)24 * kRedLdsBoxes, s, bp.nsets,
                 w.pre + bp.o_rl, w);
    if (bp.red_global)
      BBX_LAUNCH("reduce", k_reduce<false>, bp.g_rl, kRedBlock, 0, s, bp.nsets, w.pre + bp.o_rl, w);
  }
  return hipGetLastError();
}

hipError_t launch_reduce_pack(const BatchPlan& bp, const Ws& w, hipStream_t s) {
  if (!bp.reduce) return hipGetLastError();
  if (bp.g_rw > 0) {
    BBX_LAUNCH("reduce_meta", k_red_meta, bp.g_rw, kBlock, 0, s, bp.nsets, w.pre + bp.o_rw, w);
    BBX_LAUNCH("reduce_payload", k_red_payload, bp.g_rw, kBlock, 0, s, bp.nsets, w.pre + bp.o_rw, w);
    BBX_LAUNCH("reduce_perm", k_red_perm, bp.g_rw, kBlock, 0, s, bp.nsets, w.pre + bp.o_rw, w);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- decoding (version 2)

__device__ inline u128 red_read(const uint64_t* sec, uint64_t nwords, uint64_t at, uint32_t len) {
  if (len == 0) return 0;
  const uint64_t w0 = at >> 6;
  const uint32_t sh = (uint32_t)(at & 63);
  u128 v = (u128)sec[w0];
  if (w0 + 1 < nwords) v |= (u128)sec[w0 + 1] << 64;
  v >>= sh;
  if (sh + len > 128 && w0 + 2 < nwords) v |= (u128)sec[w0 + 2] << (128 - sh);
  if (len < 128) v &= (((u128)1) << len) - 1;
  return v;
}

// per sequence: widths (validated), centre codes, count; slot counts and
// payload bits for the two scans
__global__ void __launch_bounds__(kBlock) k_dec_meta2(uint64_t nseq, uint32_t dims, uint32_t mbits,
                                                      uint32_t G0, uint32_t G1, uint32_t G2,
                                                      uint64_t meta_bits, const uint8_t* stream,
                                                      LeafRec* seqs, uint64_t* bits,
                                                      uint64_t* slots, DevParams* P) {
  const uint32_t G[3] = {G0, G1, G2};
  const uint32_t Sb = dims * mbits + G0 + G1 + G2 + 32;
  const uint64_t* meta = (const uint64_t*)(stream + kHeaderBytes);
  const uint64_t nwords = (meta_bits + 63) / 64;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nseq;
       i += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t at = i * Sb;
    LeafRec rec;
    uint32_t m = 0, summ = 0;
    bool bad = false;
    for (uint32_t d = 0; d < dims; ++d, at += mbits) {
      const uint32_t md = (uint32_t)red_read(meta, nwords, at, mbits);
      if (md == 1 || md > 31 || md > G[d] + 1) bad = true;
      m |= md << (8 * d);
      summ += md;
    }
    for (uint32_t d = 0; d < 3; ++d) {
      rec.qref[d] = d < dims ? (uint32_t)red_read(meta, nwords, at, G[d]) : 0u;
      if (d < dims) at += G[d];
    }
    const uint32_t cnt = (uint32_t)red_read(meta, nwords, at, 32);
    rec.start = 0;
    rec.size = cnt;
    rec.m = m;
    rec.ref_src = 0;
    seqs[i] = rec;
    bits[i] = bad ? 0 : (uint64_t)cnt * summ;
    slots[i] = (uint64_t)cnt + 1;
    if (bad) P->status = BBX_ECORRUPT;
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_unpack2(uint64_t n, uint64_t nseq, uint32_t dims,
                                                    uint32_t layout, double w, double o0,
                                                    double o1, double o2, uint32_t G0,
                                                    uint32_t G1, uint32_t G2, uint64_t meta_bits,
                                                    uint64_t payload_bits, const LeafRec* seqs,
                                                    const uint64_t* off, const uint64_t* slots,
                                                    const uint8_t* stream, T* out, DevParams* P) {
  if (P->status != BBX_OK) return;
  const double origin[3] = {o0, o1, o2};
  const uint32_t G[3] = {G0, G1, G2};
  const uint64_t* pay = (const uint64_t*)(stream + kHeaderBytes + ((meta_bits + 63) / 64) * 8);
  const uint64_t pwords = (payload_bits + 63) / 64;
  bool corrupt = false;
  for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
       p += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t i = red_search(slots, 0, nseq, p);
    const LeafRec rec = seqs[i];
    const uint64_t j = p - slots[i];
    const uint32_t m[3] = {rec.m & 0xffu, (rec.m >> 8) & 0xffu, (rec.m >> 16) & 0xffu};
    const uint32_t sm = m[0] + m[1] + m[2];
    u128 v = 0;
    if (j > 0) v = red_read(pay, pwords, off[i] + (j - 1) * sm, sm);
    for (uint32_t d = 0; d < dims; ++d) {
      int64_t q = rec.qref[d];
      if (j > 0 && m[d]) {
        const uint32_t u = (uint32_t)(v & ((((u128)1) << m[d]) - 1));
        if (u == 0) corrupt = true;
        q += (int64_t)u - ((int64_t)1 << (m[d] - 1));
      }
      if (j > 0) v >>= m[d];
      uint32_t qq = (uint32_t)q;
      if (q < 0 || (uint64_t)q >= (1ull << G[d])) corrupt = true, qq = 0;
      const T t = (T)(origin[d] + (double)qq * w);
      if (layout == BBX_AOS)
        out[p * dims + d] = t;
      else
        out[(uint64_t)d * n + p] = t;
    }
  }
  if (corrupt) P->status = BBX_ECORRUPT;
}

hipError_t launch_decompress2(const DecompressPlan& p, const DecompressWs& w, const uint8_t* stream,
                              void* pos, hipStream_t s) {
  uint64_t g = (p.n_seq + kBlock - 1) / kBlock;
  if (g > 65536) g = 65536;
  if (g == 0) g = 1;
  BBX_LAUNCH("dec_meta2", k_dec_meta2, g, kBlock, 0, s, p.n_seq, p.dims, p.mbits, p.G[0], p.G[1],
             p.G[2], p.meta_bits, stream, w.leaves, w.leaf_bits, w.slot_start, w.params);
  // slot starts (total n), then payload offsets (total payload_bits)
  hipError_t e = launch_dec_scan(p.n_seq, w.slot_start, w.scan_part, w.params, p.n, s);
  if (e == hipSuccess) e = launch_dec_scan(p.n_seq, w.leaf_bits, w.scan_part, w.params, p.payload_bits, s);
  if (e != hipSuccess) return e;
  uint64_t gu = (p.n + kBlock - 1) / kBlock;
  if (gu > 16384) gu = 16384;
  if (p.dtype == BBX_F32)
    BBX_LAUNCH("unpack2", k_unpack2<float>, gu, kBlock, 0, s, p.n, p.n_seq, p.dims, p.layout, p.w,
               p.origin[0], p.origin[1], p.origin[2], p.G[0], p.G[1], p.G[2], p.meta_bits,
               p.payload_bits, w.leaves, w.leaf_bits, w.slot_start, stream, (float*)pos, w.params);
  else
    BBX_LAUNCH("unpack2", k_unpack2<double>, gu, kBlock, 0, s, p.n, p.n_seq, p.dims, p.layout, p.w,
               p.origin[0], p.origin[1], p.origin[2], p.G[0], p.G[1], p.G[2], p.meta_bits,
               p.payload_bits, w.leaves, w.leaf_bits, w.slot_start, stream, (double*)pos, w.params);
  return hipGetLastError();
}

}  // namespace bbx

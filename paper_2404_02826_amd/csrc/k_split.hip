// k_split.hip -- the partition under split rules 1-3, ablations of how
// Sec. 4.1's "split along one dimension at the median until at most r
// particles" is read (rule 0, the median along the axes in turn, is the
// partition of k_level.hip and k_tile.hip):
//   1  the median along the axis whose codes spread widest in the node
//      (max - min; the lowest axis on ties);
//   2  ceil(n/r) leaves: with b = ceil(n/r), leaf i holds the tree-order
//      ranks floor(i n / b) .. floor((i + 1) n / b) - 1; a node of leaves
//      [i0, i1) gives the first floor((i1 - i0) / 2) to its left child and
//      splits at the matching rank, axes in turn;
//   3  midpoint cells of the code grid (the coders Sec. 2.2 cites): the root
//      cell is [0, 2^G_d) per axis; a node of more than r particles halves
//      its cell along the axes in turn, skipping one-code-wide axes (a node
//      whose cell is one code is a leaf); codes below the midpoint go left;
//      an empty half makes no node.
// Rules 1 and 2 split at a rank k: the member of rank k in (code, index)
// order and all after it go right.  Every split is stable (both children
// keep ascending source index), so a node's members with the split code v
// go left in index order until the left child is full.
//
// Particles travel as uint4 (code x, y, z, source index) between two
// buffers.  Global levels (nodes of more than kSpLocal particles; node lists
// and counts on the device, so the launches need no host synchronization):
//   k_sp_tiles    per-node tile ranges (kSpTile particles each)
//   k_sp_extent   rule 1: per-node code min and max per axis
//   k_sp_axis     per node: split axis, rank or midpoint; selection reset
//   k_sp_hist / k_sp_pick   radix selection of the rank-k code, 8-bit digits
//   k_sp_count    per tile: codes below the split code, and equal to it
//   k_sp_scan     per node: tile offsets and children; the next level's
//                 active nodes, and the done list (leaves, and nodes of at
//                 most kSpLocal particles)
//   k_sp_scatter  the stable two-way scatter of each tile
// k_sp_local then finishes every done node inside one block (particles in
// LDS, a wavefront per node, level by level), writing each leaf's particles
// to the set's tree order and its size at its first position.  k_sp_lcount,
// k_sp_lscan and k_sp_lrec number the leaves by position (depth-first order
// is position order), and k_sp_box gives each leaf its bit box (AABB,
// reference, Eq. 2) in the state the reduction and the version-2 packer
// (k_reduce.hip) read.
//
// This path is an ablation, written for clarity over speed: each global
// level reads the particles once per pass (extents, up to four digit passes,
// counts, scatter), and the local stage selects by bitwise search.
#include "bbx_internal.h"

namespace bbx {

namespace {

struct SpCtx {
  uint4* e[2];
  uint32_t* len;
  SpNode* nodes[2];
  SpSel* sel;
  uint32_t* hist;
  uint2* tcnt;
  uint2* toff;
  SpNode* done;
  uint32_t* part;
  uint32_t* ctl;
  SpLayout L;
};

__device__ inline SpCtx sp_ctx(const SetDesc& S, const Ws& w) {
  SpCtx c;
  uint8_t* base = w.split + S.sp_off;
  c.L = sp_layout(S.n, S.sp_levels);
  c.e[0] = (uint4*)(base + c.L.e[0]);
  c.e[1] = (uint4*)(base + c.L.e[1]);
  c.len = (uint32_t*)(base + c.L.len);
  c.nodes[0] = (SpNode*)(base + c.L.nodes[0]);
  c.nodes[1] = (SpNode*)(base + c.L.nodes[1]);
  c.sel = (SpSel*)(base + c.L.sel);
  c.hist = (uint32_t*)(base + c.L.hist);
  c.tcnt = (uint2*)(base + c.L.tcnt);
  c.toff = (uint2*)(base + c.L.toff);
  c.done = (SpNode*)(base + c.L.done);
  c.part = (uint32_t*)(base + c.L.part);
  c.ctl = (uint32_t*)(base + c.L.ctl);
  return c;
}

__device__ inline uint32_t comp(const uint4 q, uint32_t d) { return d == 0 ? q.x : (d == 1 ? q.y : q.z); }

// ceil(n / r): the leaves of rule 2
__device__ inline uint64_t sp_b(const SetDesc& S) { return (S.n + S.r - 1) / S.r; }

// rule 2: the rank at which a node of leaves [i0, i1) splits (relative to
// its first particle), and its left child's last leaf + 1
__device__ inline uint32_t sp_rank2(const SetDesc& S, uint32_t i0, uint32_t i1, uint32_t* im_out) {
  const uint64_t b = sp_b(S), im = i0 + (uint64_t)(i1 - i0) / 2;
  *im_out = (uint32_t)im;
  return (uint32_t)((im * S.n) / b - ((uint64_t)i0 * S.n) / b);
}

__device__ inline bool sp_is_leaf(const SetDesc& S, uint32_t size, uint32_t i0, uint32_t i1,
                                  uint32_t pk) {
  if (S.split == 2) return i1 - i0 <= 1;
  if (size <= S.r) return true;
  if (S.split == 3) {
    bool any = false;
    for (uint32_t d = 0; d < S.dims; ++d) any = any || sp_lg(pk, d) > 0;
    return !any;
  }
  return false;
}

// rule 3: the first axis in turn from depth mod dims whose cell is wider than one code
__device__ inline uint32_t sp_axis3(const SetDesc& S, uint32_t pk) {
  const uint32_t d0 = sp_depth(pk) % S.dims;
  for (uint32_t k = 0; k < S.dims; ++k) {
    const uint32_t d = (d0 + k) % S.dims;
    if (sp_lg(pk, d) > 0) return d;
  }
  return d0;  // never: a node with no such axis is a leaf
}

// The two children of a node split at nl (the left child's size) along d.
__device__ inline void sp_children(const SetDesc& S, const SpNode& nd, uint32_t d, uint32_t nl,
                                   uint32_t buf, SpNode* L, SpNode* R) {
  *L = nd;
  *R = nd;
  const uint32_t depth = sp_depth(nd.pk) + 1;
  uint32_t pk = (nd.pk & 0x7fffu) | (buf << 16) | (depth << 24);
  L->size = nl;
  R->start = nd.start + nl;
  R->size = nd.size - nl;
  if (S.split == 2) {
    uint32_t im;
    sp_rank2(S, nd.i0, nd.i1, &im);
    L->i1 = im;
    R->i0 = im;
  }
  if (S.split == 3) {
    const uint32_t lg = sp_lg(nd.pk, d);
    pk = (pk & ~(31u << (5 * d))) | ((lg - 1) << (5 * d));
    R->lo[d] = nd.lo[d] + (1u << (lg - 1));
  }
  L->pk = pk;
  R->pk = pk;
}

// Block-wide exclusive scan (blockDim.x a multiple of 64, at most 1024);
// *total gets the sum.  Ends with a barrier, so it can be called in a loop.
__device__ inline uint32_t sp_exscan(uint32_t v, uint32_t* total) {
  __shared__ uint32_t wsum[16];
  const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const uint32_t incl = wave_incl(v);
  if (lane == 63) wsum[wv] = incl;
  __syncthreads();
  uint32_t off = 0, tot = 0;
  for (uint32_t k = 0; k < nw; ++k) {
    const uint32_t x = wsum[k];
    off += k < wv ? x : 0u;
    tot += x;
  }
  __syncthreads();
  *total = tot;
  return off + incl - v;
}

// Block-wide sum (blockDim.x a multiple of 64); every thread gets it.
__device__ inline uint32_t sp_bsum(uint32_t v) {
  uint32_t t;
  sp_exscan(v, &t);
  return t;
}

// node owning tile t of the level: the last j with tile0 <= t
__device__ inline uint32_t sp_node_of(const SpSel* sel, uint32_t na, uint32_t t) {
  uint32_t lo = 0, hi = na - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (sel[mid].tile0 <= t)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

}  // namespace

// ---------------------------------------------------------------- set-up

// The set's codes (after quantization) as uint4 with the source index, and
// the root node.
__global__ void __launch_bounds__(kBlock) k_sp_init(uint32_t s, Ws w) {
  const SetDesc& S = w.sets[s];
  const DevParams* P = w.params + s;
  if (P->status != BBX_OK || S.n == 0) return;
  const SpCtx c = sp_ctx(S, w);
  const uint8_t* keys = w.keys[0] + S.key_off;
  const uint64_t n = S.n, kst = S.kst;
  const bool k16 = P->key16 != 0;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t q[3] = {0, 0, 0};
    for (uint32_t d = 0; d < S.dims; ++d)
      q[d] = k16 ? ((const uint16_t*)keys)[d * kst + i] : ((const uint32_t*)keys)[d * kst + i];
    c.e[0][i] = make_uint4(q[0], q[1], q[2], (uint32_t)i);
    c.len[i] = 0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    SpNode r;
    r.start = 0;
    r.size = (uint32_t)n;
    r.i0 = 0;
    r.i1 = (uint32_t)sp_b(S);
    r.lo[0] = r.lo[1] = r.lo[2] = 0;
    r.pk = 0;
    for (uint32_t d = 0; d < S.dims; ++d) r.pk |= P->G[d] << (5 * d);
    const bool leaf = sp_is_leaf(S, r.size, r.i0, r.i1, r.pk);
    r.pk |= (leaf ? 1u : 0u) << 17;
    if (leaf || n <= kSpLocal) {
      c.done[0] = r;
      c.ctl[kSpDone] = 1;
      c.ctl[kSpNa0] = 0;
    } else {
      c.nodes[0][0] = r;
      c.ctl[kSpNa0] = 1;
      c.ctl[kSpDone] = 0;
    }
    c.ctl[kSpNa1] = 0;
    c.ctl[kSpTiles] = 0;
    c.ctl[kSpCovered] = 0;
  }
}

// ---------------------------------------------------------------- global levels

// One block: the level's tile list (node j's tiles are tile0 .. tile0 +
// ceil(size / kSpTile) - 1), and rule 1's extents reset.
__global__ void __launch_bounds__(1024) k_sp_tiles(uint32_t s, uint32_t level, Ws w) {
  const SetDesc& S = w.sets[s];
  const DevParams* P = w.params + s;
  if (P->status != BBX_OK || S.n == 0) return;
  const SpCtx c = sp_ctx(S, w);
  const uint32_t cur = level & 1, na = c.ctl[cur];
  uint32_t carry = 0;
  for (uint32_t j0 = 0; j0 < na; j0 += blockDim.x) {
    const uint32_t j = j0 + threadIdx.x;
    const uint32_t t = j < na ? (c.nodes[cur][j].size + kSpTile - 1) / kSpTile : 0u;
    uint32_t tot;
    const uint32_t ex = sp_exscan(t, &tot);
    if (j < na) {
      SpSel& sl = c.sel[j];
      sl.tile0 = carry + ex;
      for (uint32_t d = 0; d < 3; ++d) sl.ext[2 * d] = ~0u, sl.ext[2 * d + 1] = 0u;
    }
    carry += tot;
  }
  if (threadIdx.x == 0) c.ctl[kSpTiles] = carry;
}

// Rule 1: per node, the code min and max of every axis.
__global__ void __launch_bounds__(kBlock) k_sp_extent(uint32_t s, uint32_t level, Ws w) {
  const SetDesc& S = w.sets[s];
  const DevParams* P = w.params + s;
  if (P->status != BBX_OK || S.n == 0) return;
  const SpCtx c = sp_ctx(S, w);
  const uint32_t cur = level & 1, na = c.ctl[cur], ntiles = c.ctl[kSpTiles];
  __shared__ uint32_t red[4][6];
  for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const uint32_t j = sp_node_of(c.sel, na, t);
    const SpNode nd = c.nodes[cur][j];
    const uint32_t a = nd.start + (t - c.sel[j].tile0) * kSpTile;
    const uint32_t b = umin32(a + kSpTile, nd.start + nd.size);
    uint32_t mn[3] = {~0u, ~0u, ~0u}, mx[3] = {0, 0, 0};
    for (uint32_t i = a + threadIdx.x; i < b; i += blockDim.x) {
      const uint4 q = c.e[cur][i];
      for (uint32_t d = 0; d < 3; ++d) mn[d] = umin32(mn[d], comp(q, d)), mx[d] = umax32(mx[d], comp(q, d));
    }
    for (uint32_t d = 0; d < 3; ++d) mn[d] = wave_min_dpp(mn[d]), mx[d] = wave_max_dpp(mx[d]);
    const uint32_t wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
      for (uint32_t d = 0; d < 3; ++d) red[wv][2 * d] = mn[d], red[wv][2 * d + 1] = mx[d];
    __syncthreads();
    if (threadIdx.x < 6) {
      uint32_t v = red[0][threadIdx.x];
      for (uint32_t k = 1; k < blockDim.x / 64; ++k)
        v = (threadIdx.x & 1) ? umax32(v, red[k][threadIdx.x]) : umin32(v, red[k][threadIdx.x]);
      uint32_t* e = &c.sel[j].ext[threadIdx.x];
      if (threadIdx.x & 1)
        atomicMax(e, v);
      else
        atomicMin(e, v);
    }
    __syncthreads();
  }
}

// Per node: the split axis, and the rank to select (rules 1, 2) or the
// midpoint code (rule 3); every node's radix bins cleared.
__global__ void __launch_bounds__(kBlock) k_sp_axis(uint32_t s, uint32_t level, Ws w) {
  const SetDesc& S = w.sets[s];
  const DevParams* P = w.params + s;
  if (P->status != BBX_OK || S.n == 0) return;
  const SpCtx c = sp_ctx(S, w);
  const uint32_t cur = level & 1, na = c.ctl[cur];
  const uint64_t gt = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x, gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t j = gt; j < na; j += gs) {
    const SpNode nd = c.nodes[cur][j];
    SpSel& sl = c.sel[j];
    uint32_t d = sp_depth(nd.pk) % S.dims;
    if (S.split == 1) {  // widest extent, lowest axis on ties
      uint32_t best = 0;
      for (uint32_t a = 0; a < S.dims; ++a) {
        const uint32_t wd = sl.ext[2 * a + 1] - sl.ext[2 * a];
        if (a == 0 || wd > best) best = wd, d = a;
      }
    }
    if (S.split == 3) d = sp_axis3(S, nd.pk);
    sl.axis = d;
    sl.prefix = 0;
    if (S.split == 3) {
      sl.npass = 0;
      sl.k = nd.lo[d] + (1u << (sp_lg(nd.pk, d) - 1));
      sl.rank = 0;
    } else {
      uint32_t k = nd.size / 2, im;
      if (S.split == 2) k = sp_rank2(S, nd.i0, nd.i1, &im);
      sl.k = k;
      sl.rank = k;
      const uint32_t G = P->G[d];
      sl.npass = G > 8 ? (G + 7) / 8 : 1u;
    }
  }
  for (uint64_t x = gt; x < (uint64_t)na * 256; x += gs) c.hist[x] = 0;
}

// Radix pass p (digits of 8 bits from the top of G_d): count the digit of
// every member whose higher digits equal the prefix selected so far.
__global__ void __launch_bounds__(kBlock) k_sp_hist(uint32_t s, uint32_t level, uint32_t p, Ws w) {
  const SetDesc& S = w.sets[s];
  const DevParams* P = w.params + s;
  if (P->status != BBX_OK || S.n == 0 || S.split == 3) return;
  const SpCtx c = sp_ctx(S, w);
  const uint32_t cur = level & 1, na = c.ctl[cur], ntiles = c.ctl[kSpTiles];
  __shared__ uint32_t bins[256];
  for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const uint32_t j = sp_node_of(c.sel, na, t);
    const SpSel sl = c.sel[j];
    if (sl.npass <= p) continue;  // uniform in the block
    const SpNode nd = c.nodes[cur][j];
    const uint32_t a = nd.start + (t - sl.tile0) * kSpTile;
    const uint32_t b = umin32(a + kSpTile, nd.start + nd.size);
    const uint32_t sh = 8 * (sl.npass - 1 - p);
    bins[threadIdx.x] = 0;
    __syncthreads();
    for (uint32_t i = a + threadIdx.x; i < b; i += blockDim.x) {
      const uint32_t q = comp(c.e[cur][i], sl.axis);
      if (((uint64_t)q >> (sh + 8)) == sl.prefix) atomicAdd(&bins[(q >> sh) & 255u], 1u);
    }
    __syncthreads();
    if (bins[threadIdx.x]) atomicAdd(&c.hist[(uint64_t)j * 256 + threadIdx.x], bins[threadIdx.x]);
    __syncthreads();
  }
}

// After pass p: per node (a wavefront each) the digit holding the rank;
// the prefix gains it, the rank drops by the members below it, the bins are
// cleared for the next pass.  After the last pass the prefix is the rank-k
// code v and the rank the number of members equal to v that go left.
__global__ void __launch_bounds__(kBlock) k_sp_pick(uint32_t s, uint32_t level, uint32_t p, Ws w) {
  const SetDesc& S = w.sets[s];
  DevParams* P = w.params + s;
  if (P->status != BBX_OK || S.n == 0 || S.split == 3) return;
  const SpCtx c = sp_ctx(S, w);
  const uint32_t cur = level & 1, na = c.ctl[cur];
  const uint32_t lane = threadIdx.x & 63, wpb = blockDim.x / 64;
  for (uint32_t j = blockIdx.x * wpb + (threadIdx.x >> 6); j < na; j += gridDim.x * wpb) {
    SpSel& sl = c.sel[j];
    if (sl.npass <= p) continue;
    uint32_t* h = c.hist + (uint64_t)j * 256;
    uint32_t v[4], sum = 0;
    for (uint32_t u = 0; u < 4; ++u) v[u] = h[4 * lane + u], sum += v[u];
    const uint32_t incl = wave_incl(sum), excl = incl - sum, rank = sl.rank;
    const uint64_t hit = __ballot(excl <= rank && rank < incl);
    if (hit == 0) {
      if (lane == 0) check_failed(P, kChkSplit);
      continue;
    }
    const uint32_t L = (uint32_t)__builtin_ctzll(hit);
    uint32_t dig = 0, nr = 0;
    if (lane == L) {
      uint32_t acc = excl;
      for (uint32_t u = 0; u < 4; ++u) {
        if (rank < acc + v[u]) {
          dig = 4 * lane + u;
          nr = rank - acc;
          break;
        }
        acc += v[u];
      }
    }
    dig = (uint32_t)__builtin_amdgcn_readlane((int)dig, (int)L);
    nr = (uint32_t)__builtin_amdgcn_readlane((int)nr, (int)L);
    for (uint32_t u = 0; u < 4; ++u) h[4 * lane + u] = 0;
    if (lane == 0) {
      sl.prefix = (sl.prefix << 8) | dig;
      sl.rank = nr;
    }
  }
}

// Per tile: members below the split code (rule 3: below the midpoint), and
// (rules 1, 2) equal to it.
__global__ void __launch_bounds__(kBlock) k_sp_count(uint32_t s, uint32_t level, Ws w) {
  const SetDesc& S = w.sets[s];
  const DevParams* P = w.params + s;
  if (P->status != BBX_OK || S.n == 0) return;
  const SpCtx c = sp_ctx(S, w);
  const uint32_t cur = level & 1, na = c.ctl[cur], ntiles = c.ctl[kSpTiles];
  for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const uint32_t j = sp_node_of(c.sel, na, t);
    const SpSel sl = c.sel[j];
    const SpNode nd = c.nodes[cur][j];
    const uint32_t a = nd.start + (t - sl.tile0) * kSpTile;
    const uint32_t b = umin32(a + kSpTile, nd.start + nd.size);
    const uint32_t v = S.split == 3 ? sl.k : sl.prefix;
    uint32_t lt = 0, eq = 0;
    for (uint32_t i = a + threadIdx.x; i < b; i += blockDim.x) {
      const uint32_t q = comp(c.e[cur][i], sl.axis);
      lt += q < v ? 1u : 0u;
      eq += (S.split != 3 && q == v) ? 1u : 0u;
    }
    lt = sp_bsum(lt);
    eq = sp_bsum(eq);
    if (threadIdx.x == 0) c.tcnt[t] = make_uint2(lt, eq);
  }
}

// One block: the level-wide exclusive scan of the tile counts; per node its
// left size and children; the next level's active list and the done list.
__global__ void __launch_bounds__(1024) k_sp_scan(uint32_t s, uint32_t level, Ws w) {
  const SetDesc& S = w.sets[s];
  DevParams* P = w.params + s;
  if (P->status != BBX_OK || S.n == 0) return;
  const SpCtx c = sp_ctx(S, w);
  const uint32_t cur = level & 1, nxt = cur ^ 1, na = c.ctl[cur], ntiles = c.ctl[kSpTiles];
  uint32_t clt = 0, ceq = 0;
  for (uint32_t t0 = 0; t0 < ntiles; t0 += blockDim.x) {
    const uint32_t t = t0 + threadIdx.x;
    const uint2 v = t < ntiles ? c.tcnt[t] : make_uint2(0, 0);
    uint32_t tl, te;
    const uint32_t xl = sp_exscan(v.x, &tl), xe = sp_exscan(v.y, &te);
    if (t < ntiles) c.toff[t] = make_uint2(clt + xl, ceq + xe);
    clt += tl;
    ceq += te;
  }
  __syncthreads();
  uint32_t act = 0, dn = c.ctl[kSpDone];
  for (uint32_t j0 = 0; j0 < na; j0 += blockDim.x) {
    const uint32_t j = j0 + threadIdx.x;
    SpNode ch[2];
    uint32_t kind[2] = {0, 0};  // 0 none, 1 active, 2 done
    if (j < na) {
      SpSel& sl = c.sel[j];
      const SpNode nd = c.nodes[cur][j];
      const uint2 b = c.toff[sl.tile0];
      const uint32_t end_lt = j + 1 < na ? c.toff[c.sel[j + 1].tile0].x : clt;
      sl.base_lt = b.x;
      sl.base_eq = b.y;
      const uint32_t nl = S.split == 3 ? end_lt - b.x : sl.k;
      sl.nl = nl;
      sp_children(S, nd, sl.axis, nl, nxt, &ch[0], &ch[1]);
      for (int k = 0; k < 2; ++k) {
        if (ch[k].size == 0) continue;  // rule 3: an empty half is no node
        const bool leaf = sp_is_leaf(S, ch[k].size, ch[k].i0, ch[k].i1, ch[k].pk);
        ch[k].pk |= (leaf ? 1u : 0u) << 17;
        kind[k] = (leaf || ch[k].size <= kSpLocal) ? 2u : 1u;
      }
    }
    const uint32_t na_t = (kind[0] == 1) + (kind[1] == 1), nd_t = (kind[0] == 2) + (kind[1] == 2);
    uint32_t ta, td;
    uint32_t pa = sp_exscan(na_t, &ta), pd = sp_exscan(nd_t, &td);
    for (int k = 0; k < 2; ++k) {
      if (kind[k] == 1) {
        const uint64_t at = (uint64_t)act + pa++;
        if (at < c.L.na) c.nodes[nxt][at] = ch[k];
      } else if (kind[k] == 2) {
        const uint64_t at = (uint64_t)dn + pd++;
        if (at < c.L.dc) c.done[at] = ch[k];
      }
    }
    act += ta;
    dn += td;
  }
  if (threadIdx.x == 0) {
    if (act > c.L.na || dn > c.L.dc) {
      check_failed(P, kChkSplit);
      act = 0;
    }
    c.ctl[nxt] = act;
    c.ctl[kSpDone] = umin32(dn, (uint32_t)c.L.dc);
  }
}

// The stable two-way scatter of each tile: 8 consecutive members per thread.
__global__ void __launch_bounds__(kBlock) k_sp_scatter(uint32_t s, uint32_t level, Ws w) {
  const SetDesc& S = w.sets[s];
  const DevParams* P = w.params + s;
  if (P->status != BBX_OK || S.n == 0) return;
  const SpCtx c = sp_ctx(S, w);
  const uint32_t cur = level & 1, na = c.ctl[cur], ntiles = c.ctl[kSpTiles];
  constexpr uint32_t E = kSpTile / kBlock;
  for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const uint32_t j = sp_node_of(c.sel, na, t);
    const SpSel sl = c.sel[j];
    const SpNode nd = c.nodes[cur][j];
    const uint32_t off = (t - sl.tile0) * kSpTile;  // the tile's first member, relative to the node
    const uint32_t cnt = umin32(kSpTile, nd.size - off);
    const bool r3 = S.split == 3;
    const uint32_t v = r3 ? sl.k : sl.prefix, teq = r3 ? 0u : sl.rank;
    uint4 q[E];
    uint32_t nlt = 0, neq = 0;
    for (uint32_t u = 0; u < E; ++u) {
      const uint32_t k = threadIdx.x * E + u;
      q[u] = k < cnt ? c.e[cur][nd.start + off + k] : make_uint4(0, 0, 0, 0);
      const uint32_t x = comp(q[u], sl.axis);
      nlt += (k < cnt && x < v) ? 1u : 0u;
      neq += (k < cnt && !r3 && x == v) ? 1u : 0u;
    }
    uint32_t tot;
    const uint32_t ex = sp_exscan((nlt << 16) | neq, &tot);
    const uint2 to = c.toff[t];
    uint32_t lt_b = to.x - sl.base_lt + (ex >> 16), eq_b = to.y - sl.base_eq + (ex & 0xffffu);
    for (uint32_t u = 0; u < E; ++u) {
      const uint32_t k = threadIdx.x * E + u;
      if (k >= cnt) break;
      const uint32_t x = comp(q[u], sl.axis);
      const bool lt = x < v, eq = !r3 && x == v;
      const uint32_t left_b = lt_b + umin32(eq_b, teq);  // members before this one that go left
      const bool left = lt || (eq && eq_b < teq);
      const uint32_t dst = left ? left_b : sl.nl + (off + k - left_b);
      if (dst < nd.size) c.e[cur ^ 1][nd.start + dst] = q[u];  // always, when the counts agree
      lt_b += lt ? 1u : 0u;
      eq_b += eq ? 1u : 0u;
    }
  }
}

// ---------------------------------------------------------------- local stage

constexpr uint32_t kSpLocalBlock = 1024;
constexpr uint32_t kSpMaxActive = kSpLocal / 2;  // an active node holds at least 2 particles
constexpr size_t kSpLocalLds = 2 * sizeof(uint4) * kSpLocal + 2 * sizeof(SpNode) * kSpMaxActive;

// count of the node's members (positions [st, st + sz) of E) whose axis-d
// code is below v; uniform over the wavefront
__device__ inline uint32_t sp_wave_below(const uint4* E, uint32_t st, uint32_t sz, uint32_t d,
                                         uint32_t v) {
  uint32_t n = 0;
  for (uint32_t k0 = 0; k0 < sz; k0 += 64) {
    const uint32_t k = k0 + (threadIdx.x & 63);
    n += (uint32_t)__popcll(__ballot(k < sz && comp(E[st + k], d) < v));
  }
  return n;
}

// A leaf: its particles to the tree order, its size at its first position.
__device__ inline void sp_emit_leaf(const SpCtx& c, uint4* fin, const uint4* E, uint32_t g0,
                                    uint32_t st, uint32_t sz) {
  for (uint32_t k = threadIdx.x & 63; k < sz; k += 64) fin[g0 + st + k] = E[st + k];
  if ((threadIdx.x & 63) == 0) c.len[g0 + st] = sz;
}

// Every done node in one block: a leaf is copied out; any other node (at
// most kSpLocal particles) is loaded into LDS and split level by level, a
// wavefront per node, until every part is a leaf.
__global__ void __launch_bounds__(kSpLocalBlock) k_sp_local(uint32_t s, Ws w) {
  extern __shared__ __align__(16) uint8_t sp_dyn[];
  const SetDesc& S = w.sets[s];
  const DevParams* P = w.params + s;
  if (P->status != BBX_OK || S.n == 0) return;
  const SpCtx c = sp_ctx(S, w);
  uint4* fin = w.red_tq + S.idx_off;
  // particles of the two levels' buffers, then the two node lists
  uint4* const E0 = (uint4*)sp_dyn;
  SpNode* const N0 = (SpNode*)(sp_dyn + 2 * sizeof(uint4) * kSpLocal);
  __shared__ uint32_t s_cnt[2];
  const uint32_t ndone = c.ctl[kSpDone], lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  constexpr uint32_t W = kSpLocalBlock / 64;
  const uint32_t dims = S.dims;
  for (uint32_t i = blockIdx.x; i < ndone; i += gridDim.x) {
    const SpNode D = c.done[i];
    const uint4* src = c.e[(D.pk >> 16) & 1u] + D.start;
    if ((D.pk >> 17) & 1u) {  // a leaf (any size): copied out
      for (uint32_t k = threadIdx.x; k < D.size; k += blockDim.x) fin[D.start + k] = src[k];
      if (threadIdx.x == 0) c.len[D.start] = D.size;
      continue;
    }
    for (uint32_t k = threadIdx.x; k < D.size; k += blockDim.x) E0[k] = src[k];
    if (threadIdx.x == 0) {
      SpNode r = D;
      r.start = 0;
      N0[0] = r;
      s_cnt[0] = 1;
      s_cnt[1] = 0;
    }
    __syncthreads();
    for (uint32_t lev = 0;; ++lev) {
      const uint32_t cb = lev & 1, nb = cb ^ 1, cnt = umin32(s_cnt[cb], kSpMaxActive);
      if (cnt == 0) break;  // uniform: read after the barrier that ended the previous level
      const uint4* Ec = E0 + cb * kSpLocal;
      uint4* En = E0 + nb * kSpLocal;
      const SpNode* Nc = N0 + cb * kSpMaxActive;
      SpNode* Nn = N0 + nb * kSpMaxActive;
      for (uint32_t j = wv; j < cnt; j += W) {
        const SpNode nd = Nc[j];
        const uint32_t st = nd.start, sz = nd.size;
        uint32_t d = sp_depth(nd.pk) % dims;
        if (S.split == 1) {
          uint32_t mn[3] = {~0u, ~0u, ~0u}, mx[3] = {0, 0, 0};
          for (uint32_t k = lane; k < sz; k += 64) {
            const uint4 q = Ec[st + k];
            for (uint32_t a = 0; a < 3; ++a) mn[a] = umin32(mn[a], comp(q, a)), mx[a] = umax32(mx[a], comp(q, a));
          }
          uint32_t best = 0;
          for (uint32_t a = 0; a < dims; ++a) {
            const uint32_t wd = wave_max_dpp(mx[a]) - wave_min_dpp(mn[a]);
            if (a == 0 || wd > best) best = wd, d = a;
          }
        }
        if (S.split == 3) d = sp_axis3(S, nd.pk);
        uint32_t v, teq, nl;
        if (S.split == 3) {
          v = nd.lo[d] + (1u << (sp_lg(nd.pk, d) - 1));
          teq = 0;
          nl = sp_wave_below(Ec, st, sz, d, v);
        } else {
          uint32_t k = sz / 2, im;
          if (S.split == 2) k = sp_rank2(S, nd.i0, nd.i1, &im);
          // the rank-k code: the largest v with (members below v) <= k
          v = 0;
          for (int b = (int)P->G[d] - 1; b >= 0; --b) {
            const uint32_t cand = v | (1u << b);
            if (sp_wave_below(Ec, st, sz, d, cand) <= k) v = cand;
          }
          teq = k - sp_wave_below(Ec, st, sz, d, v);
          nl = k;
        }
        // stable partition into the other buffer, same positions
        uint32_t lb = 0, eb = 0;
        for (uint32_t k0 = 0; k0 < sz; k0 += 64) {
          const uint32_t k = k0 + lane;
          const bool ok = k < sz;
          const uint4 q = ok ? Ec[st + k] : make_uint4(0, 0, 0, 0);
          const uint32_t x = comp(q, d);
          const bool lt = ok && x < v, eq = ok && S.split != 3 && x == v;
          const uint64_t em = __ballot(eq);
          const uint32_t eqb = eb + lanes_below(em);
          const bool left = lt || (eq && eqb < teq);
          const uint64_t lm = __ballot(left);
          const uint32_t lbk = lb + lanes_below(lm);
          if (ok) En[st + (left ? lbk : nl + (k - lbk))] = q;
          lb += (uint32_t)__popcll(lm);
          eb += (uint32_t)__popcll(em);
        }
        wave_sync();
        SpNode ch[2];
        sp_children(S, nd, d, nl, 0, &ch[0], &ch[1]);
        for (int k = 0; k < 2; ++k) {
          if (ch[k].size == 0) continue;
          if (sp_is_leaf(S, ch[k].size, ch[k].i0, ch[k].i1, ch[k].pk)) {
            sp_emit_leaf(c, fin, En, D.start, ch[k].start, ch[k].size);
          } else if (lane == 0) {
            const uint32_t at = atomicAdd(&s_cnt[nb], 1u);
            if (at < kSpMaxActive) Nn[at] = ch[k];
          }
        }
      }
      __syncthreads();
      if (threadIdx.x == 0) s_cnt[cb] = 0;
      __syncthreads();
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- leaves

// per block of kSpTile positions: the leaves starting there
__global__ void __launch_bounds__(kBlock) k_sp_lcount(uint32_t s, Ws w) {
  const SetDesc& S = w.sets[s];
  const DevParams* P = w.params + s;
  if (P->status != BBX_OK || S.n == 0) return;
  const SpCtx c = sp_ctx(S, w);
  const uint64_t a = (uint64_t)blockIdx.x * kSpTile;
  uint32_t k = 0;
  for (uint64_t i = a + threadIdx.x; i < a + kSpTile && i < S.n; i += blockDim.x) k += c.len[i] ? 1u : 0u;
  k = sp_bsum(k);
  if (threadIdx.x == 0) c.part[blockIdx.x] = k;
}

// One block: exclusive scan of the block counts; the leaf count.
__global__ void __launch_bounds__(1024) k_sp_lscan(uint32_t s, uint32_t nblk, Ws w) {
  const SetDesc& S = w.sets[s];
  DevParams* P = w.params + s;
  if (P->status != BBX_OK) return;
  if (S.n == 0) {
    if (threadIdx.x == 0) P->nleaves = 0, P->nseq = 0;
    return;
  }
  const SpCtx c = sp_ctx(S, w);
  uint32_t carry = 0;
  for (uint32_t b0 = 0; b0 < nblk; b0 += blockDim.x) {
    const uint32_t b = b0 + threadIdx.x;
    const uint32_t v = b < nblk ? c.part[b] : 0u;
    uint32_t tot;
    const uint32_t ex = sp_exscan(v, &tot);
    if (b < nblk) c.part[b] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) {
    if (carry > S.n_leaves || carry == 0) {
      check_failed(P, kChkSplit);
      carry = 0;
    }
    P->nleaves = carry;
    if (!S.reduce) P->nseq = carry;  // one sequence per leaf
  }
}

// Leaf records (first position, size), numbered by position.
__global__ void __launch_bounds__(kBlock) k_sp_lrec(uint32_t s, Ws w) {
  const SetDesc& S = w.sets[s];
  const DevParams* P = w.params + s;
  if (P->status != BBX_OK || S.n == 0) return;
  const SpCtx c = sp_ctx(S, w);
  constexpr uint32_t E = kSpTile / kBlock;
  const uint64_t a = (uint64_t)blockIdx.x * kSpTile + threadIdx.x * E;
  uint32_t z[E], k = 0;
  for (uint32_t u = 0; u < E; ++u) {
    z[u] = a + u < S.n ? c.len[a + u] : 0u;
    k += z[u] ? 1u : 0u;
  }
  uint32_t tot;
  uint32_t id = c.part[blockIdx.x] + sp_exscan(k, &tot);
  LeafRec* leaves = w.leaves + S.leaf_off;
  for (uint32_t u = 0; u < E; ++u)
    if (z[u] && id < S.n_leaves) {
      LeafRec r;
      r.start = (uint32_t)(a + u);
      r.size = z[u];
      r.m = 0;
      r.qref[0] = r.qref[1] = r.qref[2] = 0;
      r.ref_src = 0;
      leaves[id++] = r;
    }
}

// Per leaf (a wavefront each): AABB, the reference (rule 0: nearest the AABB
// centre in doubled code space; rule 1: fewest Eq. 2 bits against the AABB;
// the first member on ties), widths (Eq. 2); the reduction's box state, or
// without the reduction the leaf as one sequence (reference, then the
// others in ascending index) and its payload bits.
__global__ void __launch_bounds__(kBlock) k_sp_box(uint32_t s, Ws w) {
  const SetDesc& S = w.sets[s];
  const DevParams* P = w.params + s;
  if (P->status != BBX_OK || S.n == 0) return;
  const uint64_t nl = P->nleaves;
  const uint32_t lane = threadIdx.x & 63, dims = S.dims;
  const SpCtx c = sp_ctx(S, w);
  const uint4* tq = w.red_tq + S.idx_off;
  LeafRec* leaves = w.leaves + S.leaf_off;
  uint64_t* bits = w.leaf_bits + S.leaf_off;
  uint8_t* taken = w.red_taken + S.idx_off;
  uint32_t* slot_pos = w.red_slot + S.idx_off;
  const uint64_t gw = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint64_t nw = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  for (uint64_t id = gw; id < nl; id += nw) {
    const uint32_t st = leaves[id].start, sz = leaves[id].size;
    if (sz == 0 || (uint64_t)st + sz > S.n) continue;  // never: k_sp_verify fails the set
    if (lane == 0) atomicAdd(&c.ctl[kSpCovered], sz);
    uint32_t mn[3] = {~0u, ~0u, ~0u}, mx[3] = {0, 0, 0};
    for (uint32_t k = lane; k < sz; k += 64) {
      const uint4 q = tq[st + k];
      for (uint32_t d = 0; d < 3; ++d) mn[d] = umin32(mn[d], comp(q, d)), mx[d] = umax32(mx[d], comp(q, d));
      taken[st + k] = 0;
    }
    for (uint32_t d = 0; d < 3; ++d) mn[d] = wave_min_dpp(mn[d]), mx[d] = wave_max_dpp(mx[d]);
    uint64_t bd = ~0ull;
    uint32_t bk = ~0u;
    for (uint32_t k = lane; k < sz; k += 64) {
      const uint4 q = tq[st + k];
      uint64_t dist = 0;
      for (uint32_t d = 0; d < dims; ++d) {
        const uint32_t x = comp(q, d);
        if (S.ref_rule == 1) {
          dist += red_width(umax32(x - mn[d], mx[d] - x));
        } else {
          const int64_t t = 2 * (int64_t)x - (int64_t)mn[d] - (int64_t)mx[d];
          dist += (uint64_t)(t * t);
        }
      }
      if (dist < bd) bd = dist, bk = k;  // k ascends within a lane: the first on ties
    }
    for (int o = 32; o > 0; o >>= 1) {
      const uint64_t od = __shfl_xor(bd, o);
      const uint32_t ok = (uint32_t)__shfl_xor((int)bk, o);
      if (od < bd || (od == bd && ok < bk)) bd = od, bk = ok;
    }
    const uint4 rq = tq[st + bk];
    uint32_t mp = 0, sm = 0;
    for (uint32_t d = 0; d < dims; ++d) {
      const uint32_t x = comp(rq, d);
      const uint32_t m = red_width(umax32(x - mn[d], mx[d] - x));
      mp |= m << (8 * d);
      sm += m;
    }
    if (lane == 0) {
      leaves[id].m = mp;
      leaves[id].qref[0] = rq.x;
      leaves[id].qref[1] = rq.y;
      leaves[id].qref[2] = rq.z;
      leaves[id].ref_src = rq.w;
      w.red_ref[S.leaf_off + id] = st + bk;
      w.red_ctr[S.leaf_off + id] = make_uint4(rq.x, rq.y, rq.z, mp);
      if (S.reduce) {
        w.red_key[S.leaf_off + id] = red_key(mp, dims, S.reduce, (uint32_t)id);
      } else {
        w.red_seq[S.leaf_off + id] = make_uint4(st + bk, mp, sz - 1, st);
        bits[id] = (uint64_t)(sz - 1) * sm;
        slot_pos[st] = st + bk;
      }
    }
    if (!S.reduce)
      for (uint32_t k = lane; k < sz; k += 64)
        if (k != bk) slot_pos[st + 1 + k - (k > bk ? 1u : 0u)] = st + k;
  }
  // leaf slots past the partition's leaves hold no payload
  const uint64_t gt = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x, gs = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t id = nl + gt; id < S.n_leaves; id += gs) bits[id] = 0;
}

// The partition is whole: no node left active after the last global level,
// and the leaves cover every particle once.  Otherwise the set fails (its
// packing kernels skip it).
__global__ void k_sp_verify(uint32_t s, Ws w) {
  const SetDesc& S = w.sets[s];
  DevParams* P = w.params + s;
  if (P->status != BBX_OK || S.n == 0 || threadIdx.x != 0) return;
  const SpCtx c = sp_ctx(S, w);
  if (c.ctl[S.sp_levels & 1] != 0 || c.ctl[kSpCovered] != S.n) check_failed(P, kChkSplit);
}

// ---------------------------------------------------------------- launcher

hipError_t launch_split(const BatchPlan& bp, const SetDesc* descs, const Ws& w, hipStream_t st) {
  if (!bp.split) return hipGetLastError();
  static hipError_t lds_set = hipFuncSetAttribute((const void*)k_sp_local,
                                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                                  (int)kSpLocalLds);
  if (lds_set != hipSuccess) return lds_set;
  for (uint32_t s = 0; s < bp.nsets; ++s) {
    const SetDesc& D = descs[s];
    if (!D.split || D.n == 0) {
      if (D.split)  // an empty set: no leaves, no sequences
        BBX_LAUNCH("split_leaf_scan", k_sp_lscan, 1, 1024, 0, st, s, 0u, w);
      continue;
    }
    const SpLayout L = sp_layout(D.n, D.sp_levels);
    const uint32_t gt = (uint32_t)std::min<uint64_t>(L.ta, 4096);  // tile kernels (grid-stride)
    const uint32_t gn = (uint32_t)std::min<uint64_t>((L.na + 255) / 256, 1024);
    const uint32_t gi = (uint32_t)std::min<uint64_t>((D.n + kBlock - 1) / kBlock, 8192);
    BBX_LAUNCH("split_init", k_sp_init, gi, kBlock, 0, st, s, w);
    for (uint32_t lev = 0; lev < D.sp_levels; ++lev) {
      BBX_LAUNCH("split_tiles", k_sp_tiles, 1, 1024, 0, st, s, lev, w);
      if (D.split == 1) BBX_LAUNCH("split_extent", k_sp_extent, gt, kBlock, 0, st, s, lev, w);
      BBX_LAUNCH("split_axis", k_sp_axis, gn, kBlock, 0, st, s, lev, w);
      if (D.split != 3)
        for (uint32_t p = 0; p < 4; ++p) {
          BBX_LAUNCH("split_hist", k_sp_hist, gt, kBlock, 0, st, s, lev, p, w);
          BBX_LAUNCH("split_pick", k_sp_pick, gn, kBlock, 0, st, s, lev, p, w);
        }
      BBX_LAUNCH("split_count", k_sp_count, gt, kBlock, 0, st, s, lev, w);
      BBX_LAUNCH("split_scan", k_sp_scan, 1, 1024, 0, st, s, lev, w);
      BBX_LAUNCH("split_scatter", k_sp_scatter, gt, kBlock, 0, st, s, lev, w);
    }
    const uint32_t gl = (uint32_t)std::min<uint64_t>(L.dc, 2048);
    BBX_LAUNCH("split_local", k_sp_local, gl, kSpLocalBlock, kSpLocalLds, st, s, w);
    const uint32_t nb = (uint32_t)((D.n + kSpTile - 1) / kSpTile);
    BBX_LAUNCH("split_leaf_count", k_sp_lcount, nb, kBlock, 0, st, s, w);
    BBX_LAUNCH("split_leaf_scan", k_sp_lscan, 1, 1024, 0, st, s, nb, w);
    BBX_LAUNCH("split_leaf_rec", k_sp_lrec, nb, kBlock, 0, st, s, w);
    const uint32_t gb = (uint32_t)std::min<uint64_t>((D.n_leaves + 3) / 4, 8192);
    BBX_LAUNCH("split_box", k_sp_box, gb, kBlock, 0, st, s, w);
    BBX_LAUNCH("split_verify", k_sp_verify, 1, 64, 0, st, s, w);
  }
  return hipGetLastError();
}

}  // namespace bbx

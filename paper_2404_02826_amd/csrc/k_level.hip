// k_level.hip -- the global levels of the k-d median partition (Sec. 4.1).
//
// At depth k every node is a contiguous range of the key arrays whose members
// are in ascending original index.  The node splits at the member of rank
// floor(s/2) in (q_d, index) order, d = k mod dims; that member and everything
// after it form the right child.  Because the members are stored in index
// order, "index order" is "storage order", so the split is an exact radix
// select on q_d followed by a stable partition.
//
//   k_fill_hist       zero the per-node histogram bins used by one pass
//   k_hist_mid        histogram of a high digit of q_d over the candidates
//                     (members matching the digits found so far)
//   k_select_mid      per node: pick the digit holding the median's rank
//   k_hist_last       last digit: per-chunk prefix counts + node totals
//   k_select_last     per node: the median code v, how many members equal to
//                     v go left (jeq), and each chunk's (lt, eq) base
//   k_scatter         stable partition of the keys (and source indices)
//
// Nodes of <= r particles (possible only when r exceeds the tile capacity)
// are leaves: they skip selection and are copied through.
#include "bbx_internal.h"

namespace bbx {

template <typename KT>
__device__ inline const KT* kp(const void* keys, uint64_t n, uint32_t d) {
  return (const KT*)keys + (uint64_t)d * n;
}

__device__ inline uint32_t popc64(uint64_t v) { return (uint32_t)__popcll(v); }

// Block-wide exclusive scan of one u64 per thread (256 threads); returns the
// exclusive prefix and writes the block total to *total.
__device__ inline uint64_t block_exscan_u64(uint64_t v, uint64_t* total) {
  __shared__ uint64_t wsum[kBlock / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint64_t x = v;
  for (int o = 1; o < 64; o <<= 1) {
    uint64_t y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[wv] = x;
  __syncthreads();
  uint64_t off = 0, tot = 0;
  for (int k = 0; k < kBlock / 64; ++k) {
    if (k < wv) off += wsum[k];
    tot += wsum[k];
  }
  __syncthreads();
  *total = tot;
  return off + x - v;
}

__global__ void __launch_bounds__(kBlock) k_fill_hist(uint32_t depth, uint32_t pass, uint32_t last,
                                                      uint32_t dims, uint64_t nodes,
                                                      const DevParams* P, uint32_t* hist) {
  if (P->status != BBX_OK) return;
  const DigitPlan pl = digit_plan(P->G[depth % dims]);
  if (last ? false : pass + 1 >= pl.npass) return;
  const uint32_t w = last ? pl.width[pl.npass - 1] : pl.width[pass];
  const uint64_t total = nodes << w;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (uint64_t)gridDim.x * blockDim.x)
    hist[i] = 0;
}

template <typename KT>
__device__ void hist_mid_body(uint32_t depth, uint32_t pass, uint64_t n, uint32_t dims, uint32_t r,
                              uint64_t chunks, uint32_t chunk_elems, const DevParams* P,
                              const void* keys, const NodeSel* sel, uint32_t* hist,
                              uint32_t* lh) {
  const uint32_t d = depth % dims;
  const DigitPlan pl = digit_plan(P->G[d]);
  const uint64_t j = blockIdx.x / chunks, ch = blockIdx.x % chunks;
  uint64_t st, sz;
  node_span(n, depth, j, &st, &sz);
  if (sz <= r) return;
  const uint32_t w = pl.width[pass], sh = pl.shift[pass], hs = sh + w;
  const uint32_t prefix = pass == 0 ? 0u : sel[j].prefix;
  const uint32_t nb = 1u << w, mask = nb - 1;
  for (uint32_t b = threadIdx.x; b < nb; b += blockDim.x) lh[b] = 0;
  __syncthreads();
  const KT* q = kp<KT>(keys, n, d) + st;
  const uint64_t beg = ch * (uint64_t)chunk_elems;
  const uint64_t end = beg + chunk_elems < sz ? beg + chunk_elems : sz;
  for (uint64_t p = beg + threadIdx.x; p < end; p += blockDim.x) {
    uint32_t v = q[p];
    if ((v >> hs) == prefix) atomicAdd(&lh[(v >> sh) & mask], 1u);
  }
  __syncthreads();
  for (uint32_t b = threadIdx.x; b < nb; b += blockDim.x)
    if (lh[b]) atomicAdd(&hist[(j << w) + b], lh[b]);
}

__global__ void __launch_bounds__(kBlock) k_hist_mid(uint32_t depth, uint32_t pass, uint64_t n,
                                                     uint32_t dims, uint32_t r, uint64_t chunks,
                                                     uint32_t chunk_elems, const DevParams* P,
                                                     const void* keys, const NodeSel* sel,
                                                     uint32_t* hist) {
  if (P->status != BBX_OK) return;
  if (pass + 1 >= digit_plan(P->G[depth % dims]).npass) return;
  __shared__ uint32_t lh[kHistStride];
  if (P->key16)
    hist_mid_body<uint16_t>(depth, pass, n, dims, r, chunks, chunk_elems, P, keys, sel, hist, lh);
  else
    hist_mid_body<uint32_t>(depth, pass, n, dims, r, chunks, chunk_elems, P, keys, sel, hist, lh);
}

// Per node: find the bin that holds the median's rank among nb bins.
__global__ void __launch_bounds__(kBlock) k_select_mid(uint32_t depth, uint32_t pass, uint64_t n,
                                                       uint32_t dims, uint32_t r,
                                                       const DevParams* P, NodeSel* sel,
                                                       const uint32_t* hist) {
  if (P->status != BBX_OK) return;
  const DigitPlan pl = digit_plan(P->G[depth % dims]);
  if (pass + 1 >= pl.npass) return;
  const uint64_t j = blockIdx.x;
  uint64_t st, sz;
  node_span(n, depth, j, &st, &sz);
  if (sz <= r) return;
  const uint32_t w = pl.width[pass];
  const uint32_t nb = 1u << w;
  const uint32_t rank = pass == 0 ? (uint32_t)(sz >> 1) : sel[j].rank;
  const uint32_t prefix = pass == 0 ? 0u : sel[j].prefix;
  // each thread owns 8 consecutive bins (nb <= 2048)
  uint32_t c[8];
  uint64_t mine = 0;
  for (int k = 0; k < 8; ++k) {
    uint32_t b = threadIdx.x * 8 + k;
    c[k] = b < nb ? hist[(j << w) + b] : 0u;
    mine += c[k];
  }
  uint64_t tot;
  uint64_t cum = block_exscan_u64(mine, &tot);
  for (int k = 0; k < 8; ++k) {
    if (cum <= rank && rank < cum + c[k]) {
      NodeSel s;
      s.prefix = (prefix << w) | (threadIdx.x * 8 + k);
      s.rank = rank - (uint32_t)cum;
      s.v = 0;
      s.jeq = 0;
      sel[j] = s;
    }
    cum += c[k];
  }
}

template <typename KT>
__device__ void hist_last_body(uint32_t depth, uint64_t n, uint32_t dims, uint32_t r,
                               uint64_t chunks, uint32_t chunk_elems, const DevParams* P,
                               const void* keys, const NodeSel* sel, uint32_t* hist,
                               uint32_t* rows, uint32_t* lh) {
  const uint32_t d = depth % dims;
  const DigitPlan pl = digit_plan(P->G[d]);
  const uint32_t pass = pl.npass - 1;
  const uint64_t j = blockIdx.x / chunks, ch = blockIdx.x % chunks;
  uint64_t st, sz;
  node_span(n, depth, j, &st, &sz);
  if (sz <= r) return;
  const uint32_t w = pl.width[pass], sh = pl.shift[pass], hs = sh + w;
  const uint32_t prefix = pass == 0 ? 0u : sel[j].prefix;
  const uint32_t nb = 1u << w, mask = nb - 1;
  lh[threadIdx.x] = 0;
  __syncthreads();
  const KT* q = kp<KT>(keys, n, d) + st;
  const uint64_t beg = ch * (uint64_t)chunk_elems;
  const uint64_t end = beg + chunk_elems < sz ? beg + chunk_elems : sz;
  uint32_t below = 0;
  for (uint64_t p = beg + threadIdx.x; p < end; p += blockDim.x) {
    uint32_t v = q[p];
    uint32_t hi = v >> hs;
    if (hi == prefix)
      atomicAdd(&lh[(v >> sh) & mask], 1u);
    else if (hi < prefix)
      ++below;
  }
  __syncthreads();
  uint32_t cnt = threadIdx.x < nb ? lh[threadIdx.x] : 0u;
  uint64_t tot;
  uint64_t ex = block_exscan_u64(((uint64_t)below << 32) | cnt, &tot);
  uint32_t* row = rows + (uint64_t)blockIdx.x * kRowStride;
  row[threadIdx.x] = (uint32_t)ex;  // candidates with a smaller last digit
  if (threadIdx.x == 0) {
    row[256] = (uint32_t)tot;          // all candidates of the chunk
    row[257] = (uint32_t)(tot >> 32);  // members below the prefix
  }
  if (threadIdx.x < nb && cnt) atomicAdd(&hist[(j << w) + threadIdx.x], cnt);
}

__global__ void __launch_bounds__(kBlock) k_hist_last(uint32_t depth, uint64_t n, uint32_t dims,
                                                      uint32_t r, uint64_t chunks,
                                                      uint32_t chunk_elems, const DevParams* P,
                                                      const void* keys, const NodeSel* sel,
                                                      uint32_t* hist, uint32_t* rows) {
  if (P->status != BBX_OK) return;
  __shared__ uint32_t lh[kBlock];
  if (P->key16)
    hist_last_body<uint16_t>(depth, n, dims, r, chunks, chunk_elems, P, keys, sel, hist, rows, lh);
  else
    hist_last_body<uint32_t>(depth, n, dims, r, chunks, chunk_elems, P, keys, sel, hist, rows, lh);
}

__global__ void __launch_bounds__(kBlock) k_select_last(uint32_t depth, uint64_t n, uint32_t dims,
                                                        uint32_t r, uint64_t chunks,
                                                        const DevParams* P, NodeSel* sel,
                                                        const uint32_t* hist, const uint32_t* rows,
                                                        uint32_t* chunk_base) {
  if (P->status != BBX_OK) return;
  const DigitPlan pl = digit_plan(P->G[depth % dims]);
  const uint32_t pass = pl.npass - 1;
  const uint64_t j = blockIdx.x;
  uint64_t st, sz;
  node_span(n, depth, j, &st, &sz);
  if (sz <= r) return;
  const uint32_t w = pl.width[pass];
  const uint32_t nb = 1u << w;
  const uint32_t rank = pass == 0 ? (uint32_t)(sz >> 1) : sel[j].rank;
  const uint32_t prefix = pass == 0 ? 0u : sel[j].prefix;
  __shared__ uint32_t s_b, s_jeq;
  if (threadIdx.x == 0) s_b = 0, s_jeq = 0;  // ordered before the finder by the scan's barriers
  uint32_t c = threadIdx.x < nb ? hist[(j << w) + threadIdx.x] : 0u;
  uint64_t tot;
  uint64_t cum = block_exscan_u64(c, &tot);
  if (threadIdx.x < nb && cum <= rank && rank < cum + c) {
    s_b = threadIdx.x;
    s_jeq = rank - (uint32_t)cum;
  }
  __syncthreads();
  const uint32_t b = s_b, jeq = s_jeq;
  if (threadIdx.x == 0) {
    NodeSel s;
    s.prefix = prefix;
    s.rank = rank;
    s.v = (prefix << w) | b;
    s.jeq = jeq;
    sel[j] = s;
  }
  // per-chunk counts of members below v (lt) and equal to v (eq), then an
  // exclusive scan over the node's chunks (both packed in one u64)
  const uint64_t per = (chunks + kBlock - 1) / kBlock;
  const uint64_t c0 = threadIdx.x * per;
  uint64_t mine = 0;
  for (uint64_t k = 0; k < per; ++k) {
    uint64_t ch = c0 + k;
    if (ch >= chunks) break;
    const uint32_t* row = rows + (j * chunks + ch) * kRowStride;
    uint64_t lt = (uint64_t)row[257] + row[b];
    uint64_t eq = (uint64_t)row[b + 1] - row[b];
    mine += (eq << 32) | lt;
  }
  uint64_t run = block_exscan_u64(mine, &tot);
  for (uint64_t k = 0; k < per; ++k) {
    uint64_t ch = c0 + k;
    if (ch >= chunks) break;
    const uint32_t* row = rows + (j * chunks + ch) * kRowStride;
    uint64_t lt = (uint64_t)row[257] + row[b];
    uint64_t eq = (uint64_t)row[b + 1] - row[b];
    chunk_base[(j * chunks + ch) * 2 + 0] = (uint32_t)run;
    chunk_base[(j * chunks + ch) * 2 + 1] = (uint32_t)(run >> 32);
    run += (eq << 32) | lt;
  }
}

template <typename KT>
__device__ void scatter_body(uint32_t depth, uint64_t n, uint32_t dims, uint32_t r,
                             uint64_t chunks, uint32_t chunk_elems, DevParams* P,
                             const NodeSel* sel, const uint32_t* chunk_base, const void* src,
                             void* dst, const uint32_t* isrc, uint32_t* idst) {
  const uint32_t d = depth % dims;
  const uint64_t j = blockIdx.x / chunks, ch = blockIdx.x % chunks;
  uint64_t st, sz;
  node_span(n, depth, j, &st, &sz);
  const uint64_t beg = ch * (uint64_t)chunk_elems;
  if (beg >= sz) return;
  const uint64_t end = beg + chunk_elems < sz ? beg + chunk_elems : sz;
  const KT* s0 = (const KT*)src;
  KT* d0 = (KT*)dst;
  if (sz <= r) {  // leaf: copy through
    for (uint64_t p = beg + threadIdx.x; p < end; p += blockDim.x) {
      for (uint32_t dd = 0; dd < dims; ++dd) d0[(uint64_t)dd * n + st + p] = s0[(uint64_t)dd * n + st + p];
      if (isrc) idst[st + p] = isrc[st + p];
    }
    return;
  }
  const NodeSel s = sel[j];
  const uint32_t v = s.v, jeq = s.jeq;
  const uint64_t half = sz >> 1;
  uint64_t lt_run = chunk_base[blockIdx.x * 2 + 0];
  uint64_t eq_run = chunk_base[blockIdx.x * 2 + 1];
  __shared__ uint32_t wl[2][kBlock / 64], we[2][kBlock / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint64_t below_me = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const KT* q = s0 + (uint64_t)d * n + st;
  int it = 0;
  for (uint64_t base = beg; base < end; base += blockDim.x, ++it) {
    const uint64_t p = base + threadIdx.x;
    const bool active = p < end;
    const uint32_t key = active ? (uint32_t)q[p] : 0u;
    const bool lt = active && key < v;
    const bool eq = active && key == v;
    const uint64_t mlt = __ballot(lt), meq = __ballot(eq);
    const int buf = it & 1;
    if (lane == 0) {
      wl[buf][wv] = popc64(mlt);
      we[buf][wv] = popc64(meq);
    }
    __syncthreads();
    uint64_t ol = 0, oe = 0, tl = 0, te = 0;
    for (int k = 0; k < kBlock / 64; ++k) {
      if (k < wv) ol += wl[buf][k], oe += we[buf][k];
      tl += wl[buf][k];
      te += we[buf][k];
    }
    if (active) {
      const uint64_t L = lt_run + ol + popc64(mlt & below_me);
      const uint64_t E = eq_run + oe + popc64(meq & below_me);
      const uint64_t lb = L + (E < jeq ? E : (uint64_t)jeq);
      const bool left = lt || (eq && E < jeq);
      const uint64_t dest = left ? lb : half + (p - lb);
      if (dest >= sz) {  // inconsistent counts: never expected; refuse to write out of the node
        P->status = BBX_EHIP;
        continue;
      }
      for (uint32_t dd = 0; dd < dims; ++dd)
        d0[(uint64_t)dd * n + st + dest] = dd == d ? (KT)key : s0[(uint64_t)dd * n + st + p];
      if (isrc) idst[st + dest] = isrc[st + p];
    }
    lt_run += tl;
    eq_run += te;
  }
}

__global__ void __launch_bounds__(kBlock) k_scatter(uint32_t depth, uint64_t n, uint32_t dims,
                                                    uint32_t r, uint64_t chunks,
                                                    uint32_t chunk_elems, DevParams* P,
                                                    const NodeSel* sel,
                                                    const uint32_t* chunk_base, const void* src,
                                                    void* dst, const uint32_t* isrc,
                                                    uint32_t* idst) {
  if (P->status != BBX_OK) return;
  if (P->key16)
    scatter_body<uint16_t>(depth, n, dims, r, chunks, chunk_elems, P, sel, chunk_base, src, dst,
                           isrc, idst);
  else
    scatter_body<uint32_t>(depth, n, dims, r, chunks, chunk_elems, P, sel, chunk_base, src, dst,
                           isrc, idst);
}

LevelShape level_shape(const CompressPlan& p, uint32_t depth) {
  LevelShape sh;
  sh.depth = depth;
  sh.nodes = 1ull << depth;
  const uint64_t maxsz = (p.n + sh.nodes - 1) >> depth;  // ceil(n / 2^depth)
  const uint64_t target_blocks = 4096;
  uint64_t cpn = (target_blocks + sh.nodes - 1) / sh.nodes;
  if (cpn == 0) cpn = 1;
  uint64_t elems = (maxsz + cpn - 1) / cpn;
  uint64_t iters = (elems + kBlock - 1) / kBlock;
  if (iters < 16) iters = 16;
  sh.iters = (uint32_t)iters;
  const uint64_t ce = iters * kBlock;
  sh.chunks = (maxsz + ce - 1) / ce;
  if (sh.chunks == 0) sh.chunks = 1;
  return sh;
}

hipError_t launch_levels(const CompressPlan& p, const CompressWs& w, hipStream_t s,
                         int* final_buf) {
  int cur = 0;
  for (uint32_t k = 0; k < p.global_levels; ++k) {
    const LevelShape sh = level_shape(p, k);
    const uint64_t grid = sh.nodes * sh.chunks;
    const uint32_t ce = sh.iters * kBlock;
    const uint32_t fill_grid = 1024;
    for (uint32_t pass = 0; pass < 2; ++pass) {
      BBX_LAUNCH("level_fill", k_fill_hist, fill_grid, kBlock, 0, s, k, pass, 0u, p.dims,
                 sh.nodes, w.params, w.hist);
      BBX_LAUNCH("level_hist_mid", k_hist_mid, grid, kBlock, 0, s, k, pass, p.n, p.dims, p.r,
                 sh.chunks, ce, w.params, w.keys[cur], w.sel, w.hist);
      BBX_LAUNCH("level_select_mid", k_select_mid, sh.nodes, kBlock, 0, s, k, pass, p.n, p.dims,
                 p.r, w.params, w.sel, w.hist);
    }
    BBX_LAUNCH("level_fill", k_fill_hist, fill_grid, kBlock, 0, s, k, 0u, 1u, p.dims, sh.nodes,
               w.params, w.hist);
    BBX_LAUNCH("level_hist_last", k_hist_last, grid, kBlock, 0, s, k, p.n, p.dims, p.r, sh.chunks,
               ce, w.params, w.keys[cur], w.sel, w.hist, w.rows);
    BBX_LAUNCH("level_select_last", k_select_last, sh.nodes, kBlock, 0, s, k, p.n, p.dims, p.r,
               sh.chunks, w.params, w.sel, w.hist, w.rows, w.chunk_base);
    BBX_LAUNCH("level_scatter", k_scatter, grid, kBlock, 0, s, k, p.n, p.dims, p.r, sh.chunks, ce,
               w.params, w.sel, w.chunk_base, w.keys[cur], w.keys[cur ^ 1],
               p.track_idx ? w.idx[cur] : nullptr, p.track_idx ? w.idx[cur ^ 1] : nullptr);
    cur ^= 1;
  }
  *final_buf = cur;
  return hipGetLastError();
}

}  // namespace bbx

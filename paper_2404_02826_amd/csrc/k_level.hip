// k_level.hip -- the global levels of the k-d median partition (Sec. 4.1),
// for every set of a batch that still has nodes above the tile capacity.
//
// At depth k every node is a contiguous range of the set's code arrays whose
// members are in ascending original index.  The node splits at the member of
// rank floor(s/2) in (q_d, index) order, d = k mod dims; that member and
// everything after it form the right child.  Because the members are stored
// in index order, "index order" is "storage order", so the split is an exact
// radix select on q_d followed by a stable partition.
//
//   (the histogram bins are zeroed once per call before quantization, which
//   also builds the first-digit histogram of depth 0; every select kernel
//   re-zeroes the bins it reads)
//   k_hist_mid     histogram of a further high digit over the candidates
//                  (members matching the digits found so far)
//   k_select_mid   per node: the digit holding the median's rank
//   k_hist_last    last digit: per-chunk prefix counts + node totals
//   k_select_last  per node: the median code v, how many members equal to v
//                  go left (jeq), and each chunk's (lt, eq) base
//   k_scatter      stable partition of the codes (and source indices); also
//                  builds the next level's first-digit histogram, so that
//                  level needs no separate pass over its codes for it
//   k_level_local  a level whose nodes each fit one block: median and
//                  partition per block, no global histograms
//   k_level_wave   a level of nodes of <= 4096 members: one wavefront each
//   k_level_fused  two levels in one in-place pass with the node in
//                  registers (the last four levels above the tile stage)
//
// Streaming kernels keep 8 loads in flight per thread (rows of 256 elements,
// 8 rows per group) and synchronize once per 2048 elements.
// Nodes of <= r particles (possible only when r exceeds the tile capacity)
// are leaves: they skip selection and are copied through.
#include "bbx_internal.h"

namespace bbx {

__device__ inline uint32_t popc64(uint64_t v) { return (uint32_t)__popcll(v); }

// element d of a 3-array held in registers (d is wave-uniform; no dynamic indexing)
__device__ inline uint32_t pick3(const uint32_t* k, uint32_t d) {
  return d == 0 ? k[0] : (d == 1 ? k[1] : k[2]);
}

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

// Which optional mid passes run: flag [k][p] is set when some set has a
// global level k whose code needs more than p + 1 digit passes.  Kernels of a
// pass nobody needs exit at their first instruction.
__global__ void __launch_bounds__(kBlock) k_pass_flags(uint32_t nsets, const SetDesc* sets,
                                                       const DevParams* params,
                                                       uint32_t* pass_need) {
  for (uint32_t i = threadIdx.x; i < 4 * kMaxDepth; i += blockDim.x) pass_need[i] = 0;
  __syncthreads();
  for (uint32_t s = threadIdx.x; s < nsets; s += blockDim.x) {
    const SetDesc& S = sets[s];
    const DevParams& P = params[s];
    if (P.status != BBX_OK) continue;
    for (uint32_t k = 0; k < S.gl && k < (uint32_t)kMaxDepth; ++k) {
      if (level_is_local(S.n, k)) break;  // local levels form a suffix
      if (level_fused(S, k)) continue;
      const uint32_t np = digit_plan(P.G[k % S.dims]).npass;
      for (uint32_t p = 0; p + 1 < np && p < 4; ++p) atomicOr(&pass_need[k * 4 + p], 1u);
    }
  }
}


// The block's set, local block index and level shape.
struct LevelCtx {
  uint32_t s;
  uint64_t lb;
  LevelShape sh;
};

__device__ inline LevelCtx level_ctx(uint32_t nsets, const uint64_t* pre, const SetDesc* sets,
                                     uint32_t depth, uint64_t vb) {
  LevelCtx c;
  c.s = find_set(pre, nsets, vb);
  c.lb = vb - pre[c.s];
  c.sh = level_shape(sets[c.s].n, depth, sets[c.s].level_blocks);
  return c;
}
__device__ inline LevelCtx level_ctx(uint32_t nsets, const uint64_t* pre, const SetDesc* sets,
                                     uint32_t depth) {
  return level_ctx(nsets, pre, sets, depth, blockIdx.x);
}

// The buffers a level of set S reads (a, ia) and writes (b, ib): the launch
// passes buffer 0 then buffer 1, and paired levels before `depth` shift
// which one holds the codes.
__device__ inline void level_bufs(const SetDesc& S, uint32_t depth, uint8_t*& a, uint8_t*& b,
                                  uint32_t*& ia, uint32_t*& ib) {
  if (key_buf(S, depth)) {
    uint8_t* t = a;
    a = b;
    b = t;
    uint32_t* u = ia;
    ia = ib;
    ib = u;
  }
}

// Calls f(code) for every code of axis[A, B) (absolute element indices) with
// 16-byte loads, U of them in flight per thread.  The axis array is 16-byte
// aligned and readable up to B rounded up to 16 bytes.
template <typename KT, typename F>
__device__ inline void scan_codes(const KT* axis, uint64_t A, uint64_t B, F&& f) {
  constexpr uint32_t V = 16 / sizeof(KT);
  constexpr uint32_t U = 4;
  constexpr uint64_t STEP = (uint64_t)kBlock * V * U;
  for (uint64_t W = A & ~(uint64_t)(V - 1); W < B; W += STEP) {
    union {
      uint4 v;
      KT e[V];
    } u[U];
    if (W >= A && W + STEP <= B) {  // interior step: no bounds checks
      const uint4* a = (const uint4*)(axis + W) + threadIdx.x;
#pragma unroll
      for (uint32_t i = 0; i < U; ++i) u[i].v = a[i * kBlock];
#pragma unroll
      for (uint32_t i = 0; i < U; ++i)
#pragma unroll
        for (uint32_t k = 0; k < V; ++k) f((uint32_t)u[i].e[k]);
      continue;
    }
#pragma unroll
    for (uint32_t i = 0; i < U; ++i) {
      const uint64_t e0 = W + ((uint64_t)i * kBlock + threadIdx.x) * V;
      u[i].v = make_uint4(0, 0, 0, 0);
      if (e0 < B && e0 + V > A) u[i].v = *(const uint4*)(axis + e0);
    }
#pragma unroll
    for (uint32_t i = 0; i < U; ++i) {
      const uint64_t e0 = W + ((uint64_t)i * kBlock + threadIdx.x) * V;
#pragma unroll
      for (uint32_t k = 0; k < V; ++k) {
        const uint64_t e = e0 + k;
        if (e >= A && e < B) f((uint32_t)u[i].e[k]);
      }
    }
  }
}

template <typename KT>
__device__ void hist_mid_body(uint32_t depth, uint32_t pass, const SetDesc& S, const DevParams* P,
                              const LevelCtx& c, const uint8_t* keys, const NodeSel* sel,
                              uint32_t* hist, uint32_t* lh) {
  const uint64_t n = S.n;
  const uint32_t d = depth % S.dims;
  const DigitPlan pl = digit_plan(P->G[d]);
  const uint64_t j = c.lb / c.sh.chunks, ch = c.lb % c.sh.chunks;
  uint64_t st, sz;
  node_span(n, depth, j, &st, &sz);
  if (sz <= S.r) return;
  const uint32_t w = dp_width(pl, pass), sh = dp_shift(pl, pass), hs = sh + w;
  const uint32_t prefix = sel[j].prefix;
  const uint32_t nb = 1u << w, mask = nb - 1;
  lh[threadIdx.x] = 0;
  __syncthreads();
  const KT* q = (const KT*)keys + (uint64_t)d * S.kst;
  const uint64_t beg64 = ch * (uint64_t)c.sh.chunk_elems;
  const uint64_t A = st + (beg64 < sz ? beg64 : sz);
  const uint64_t B = st + (beg64 + c.sh.chunk_elems < sz ? beg64 + c.sh.chunk_elems : sz);
  scan_codes(q, A, B, [&](uint32_t v) {
    if ((v >> hs) == prefix) atomicAdd(&lh[(v >> sh) & mask], 1u);
  });
  __syncthreads();
  if (threadIdx.x < nb && lh[threadIdx.x]) atomicAdd(&hist[(j << 8) + threadIdx.x], lh[threadIdx.x]);
}

// passes >= 1 of a code with more than two digits (pass 0 is built by the
// previous scatter, or by the quantize pass at depth 0)
__global__ void __launch_bounds__(kBlock) k_hist_mid(uint32_t depth, uint32_t pass, uint32_t nsets,
                                                     const uint64_t* pre, const SetDesc* sets,
                                                     const DevParams* params, uint8_t* keys0,
                                                     uint8_t* keys1, const NodeSel* sel0,
                                                     uint32_t* hist0, const uint32_t* pass_need) {
  if (!pass_need[depth * 4 + pass]) return;
  __shared__ uint32_t lh[kHistBins];
  const uint64_t total = pre[nsets];
  for (uint64_t vb = blockIdx.x; vb < total; vb += gridDim.x) {  // block-uniform
    const LevelCtx c = level_ctx(nsets, pre, sets, depth, vb);
    const SetDesc& S = sets[c.s];
    const DevParams* P = params + c.s;
    if (P->status != BBX_OK) continue;
    if (level_is_local(S.n, depth) || pair_second(S, depth)) continue;
    if (pass + 1 >= digit_plan(P->G[depth % S.dims]).npass) continue;
    const uint8_t* keys = (key_buf(S, depth) ? keys1 : keys0) + S.key_off;
    if (P->key16)
      hist_mid_body<uint16_t>(depth, pass, S, P, c, keys, sel_level(S, depth, sel0), hist0 + S.hist_off, lh);
    else
      hist_mid_body<uint32_t>(depth, pass, S, P, c, keys, sel_level(S, depth, sel0), hist0 + S.hist_off, lh);
  }
}

// Per node: find the bin that holds the median's rank, then clear the bins.
// One wavefront per node (4 bins per lane); the grid is capped and strides
// over the level's nodes, so passes that a code does not need cost little.
__global__ void __launch_bounds__(kBlock) k_select_mid(uint32_t depth, uint32_t pass, uint32_t virt,
                                                       uint32_t nsets, const uint64_t* pre,
                                                       const SetDesc* sets,
                                                       const DevParams* params, NodeSel* sel0,
                                                       uint32_t* hist0, const uint32_t* pass_need) {
  if (!pass_need[depth * 4 + pass]) return;
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t total = pre[nsets];
  constexpr uint32_t wpb = kBlock / 64;
  for (uint64_t gn = (uint64_t)blockIdx.x * wpb + (threadIdx.x >> 6); gn < total;
       gn += (uint64_t)gridDim.x * wpb) {
    const uint32_t s = find_set(pre, nsets, gn);
    const SetDesc& S = sets[s];
    const DevParams* P = params + s;
    if (P->status != BBX_OK) continue;
    if (level_is_local(S.n, depth)) continue;
    // virt: the second level of a pair, selected before its data moves
    if (virt ? !(depth > 0 && pair_first(S, depth - 1)) : pair_second(S, depth)) continue;
    const DigitPlan pl = digit_plan(P->G[depth % S.dims]);
    if (pass + 1 >= pl.npass) continue;
    const uint64_t j = gn - pre[s];
    uint64_t st, sz;
    node_span(S.n, depth, j, &st, &sz);
    if (sz <= S.r) continue;
    NodeSel* sel = sel_level(S, depth, sel0);
    uint32_t* hist = hist0 + S.hist_off + (j << 8);
    const uint32_t w = dp_width(pl, pass);
    const uint32_t nb = 1u << w;
    const uint32_t rank = pass == 0 ? (uint32_t)(sz >> 1) : sel[j].rank;
    const uint32_t prefix = pass == 0 ? 0u : sel[j].prefix;
    uint32_t c[4], mine = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t b = lane * 4 + k;
      c[k] = b < nb ? hist[b] : 0u;
      mine += c[k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (c[k]) hist[lane * 4 + k] = 0;
    uint32_t cum = wave_incl(mine) - mine;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (cum <= rank && rank < cum + c[k]) {
        NodeSel ns;
        ns.prefix = (prefix << w) | (lane * 4 + k);
        ns.rank = rank - cum;
        ns.v = 0;
        ns.jeq = 0;
        sel[j] = ns;
      }
      cum += c[k];
    }
  }
}


template <typename KT>
__device__ void hist_last_body(uint32_t depth, const SetDesc& S, const DevParams* P,
                               const LevelCtx& c, const uint8_t* keys, const NodeSel* sel,
                               uint32_t* hist, uint32_t* rows, uint32_t* lh) {
  const uint64_t n = S.n;
  const uint32_t d = depth % S.dims;
  const DigitPlan pl = digit_plan(P->G[d]);
  const uint32_t pass = pl.npass - 1;
  const uint64_t j = c.lb / c.sh.chunks, ch = c.lb % c.sh.chunks;
  uint64_t st, sz;
  node_span(n, depth, j, &st, &sz);
  if (sz <= S.r) return;
  const uint32_t w = dp_width(pl, pass), sh = dp_shift(pl, pass), hs = sh + w;
  const uint32_t prefix = pass == 0 ? 0u : sel[j].prefix;
  const uint32_t nb = 1u << w, mask = nb - 1;
  lh[threadIdx.x] = 0;
  __syncthreads();
  const KT* q = (const KT*)keys + (uint64_t)d * S.kst;
  const uint64_t beg64 = ch * (uint64_t)c.sh.chunk_elems;
  const uint64_t A = st + (beg64 < sz ? beg64 : sz);
  const uint64_t B = st + (beg64 + c.sh.chunk_elems < sz ? beg64 + c.sh.chunk_elems : sz);
  uint32_t below = 0;
  scan_codes(q, A, B, [&](uint32_t v) {
    const uint32_t hi = v >> hs;
    below += hi < prefix ? 1u : 0u;
    if (hi == prefix) atomicAdd(&lh[(v >> sh) & mask], 1u);
  });
  __syncthreads();
  const uint32_t cnt = threadIdx.x < nb ? lh[threadIdx.x] : 0u;
  uint64_t tot;
  const uint64_t ex = block_exscan_u64(((uint64_t)below << 32) | cnt, &tot);
  uint32_t* row = rows + c.lb * kRowStride;
  row[threadIdx.x] = (uint32_t)ex;  // candidates with a smaller last digit
  if (threadIdx.x == 0) {
    row[256] = (uint32_t)tot;          // all candidates of the chunk
    row[257] = (uint32_t)(tot >> 32);  // members below the prefix
  }
  if (threadIdx.x < nb && cnt) atomicAdd(&hist[(j << 8) + threadIdx.x], cnt);
}

__global__ void __launch_bounds__(kBlock) k_hist_last(uint32_t depth, uint32_t nsets,
                                                      const uint64_t* pre, const SetDesc* sets,
                                                      const DevParams* params, uint8_t* keys0,
                                                      uint8_t* keys1, const NodeSel* sel0,
                                                      uint32_t* hist0, uint32_t* rows0) {
  const LevelCtx c = level_ctx(nsets, pre, sets, depth);
  const SetDesc& S = sets[c.s];
  const DevParams* P = params + c.s;
  if (P->status != BBX_OK) return;
  if (level_is_local(S.n, depth) || pair_second(S, depth)) return;
  __shared__ uint32_t lh[kBlock];
  const uint8_t* keys = (key_buf(S, depth) ? keys1 : keys0) + S.key_off;
  if (P->key16)
    hist_last_body<uint16_t>(depth, S, P, c, keys, sel_level(S, depth, sel0), hist0 + S.hist_off,
                             rows0 + S.rows_off, lh);
  else
    hist_last_body<uint32_t>(depth, S, P, c, keys, sel_level(S, depth, sel0), hist0 + S.hist_off,
                             rows0 + S.rows_off, lh);
}

// One wavefront: the last digit b holding the node's median rank among the
// node's 2^w last-digit bins (re-zeroed after the read) and the rank jeq of
// the median among the members equal to it.  False when the bins hold fewer
// members than the rank (inconsistent counts, never expected).
__device__ inline bool last_digit_of(uint32_t* hist, uint32_t nb, uint32_t rank, uint32_t* b_out,
                                     uint32_t* jeq_out) {
  const uint32_t lane = threadIdx.x & 63;
  uint32_t c[4], mine = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t b = lane * 4 + k;
    c[k] = b < nb ? hist[b] : 0u;
    mine += c[k];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (c[k]) hist[lane * 4 + k] = 0;
  uint32_t cum = wave_incl(mine) - mine;
  uint32_t fb = 0, fj = 0;
  bool found = false;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (cum <= rank && rank < cum + c[k]) found = true, fb = lane * 4 + k, fj = rank - cum;
    cum += c[k];
  }
  const uint64_t fm = __ballot(found);
  if (fm == 0) return false;
  const int fl = __ffsll((unsigned long long)fm) - 1;  // exactly one lane finds the rank
  *b_out = (uint32_t)__builtin_amdgcn_readlane((int)fb, fl);
  *jeq_out = (uint32_t)__builtin_amdgcn_readlane((int)fj, fl);
  return true;
}

// The node of a last-digit select, or false when the set or node has none.
struct LastSel {
  const SetDesc* S;
  DevParams* P;
  uint64_t j, chunks;
  uint32_t rank, prefix, w;
};
// virt: the second level of a pair, whose nodes still lie inside their
// parents (the parent level's chunks, one row per child and chunk)
__device__ inline bool last_sel_node(uint32_t depth, uint32_t virt, uint32_t nsets,
                                     const uint64_t* pre, const SetDesc* sets,
                                     const DevParams* params, const NodeSel* sel0, uint64_t gn,
                                     LastSel* o) {
  const uint32_t s = find_set(pre, nsets, gn);
  const SetDesc& S = sets[s];
  const DevParams* P = params + s;
  if (P->status != BBX_OK) return false;
  if (level_is_local(S.n, depth)) return false;
  if (virt ? !(depth > 0 && pair_first(S, depth - 1)) : pair_second(S, depth)) return false;
  const DigitPlan pl = digit_plan(P->G[depth % S.dims]);
  const uint32_t pass = pl.npass - 1;
  const uint64_t j = gn - pre[s];
  uint64_t st, sz;
  node_span(S.n, depth, j, &st, &sz);
  if (sz <= S.r) return false;
  o->S = &S;
  o->P = (DevParams*)P;
  o->j = j;
  o->chunks = level_shape(S.n, virt ? depth - 1 : depth, S.level_blocks).chunks;
  o->w = dp_width(pl, pass);
  o->rank = pass == 0 ? (uint32_t)(sz >> 1) : sel_level(S, depth, sel0)[j].rank;
  o->prefix = pass == 0 ? 0u : sel_level(S, depth, sel0)[j].prefix;
  return true;
}

// Per node: the median code v and how many members equal to v go left, then
// each chunk's (lt, eq) base by an exclusive scan over the node's chunks.
// One wavefront per node, capped grid striding over the nodes (levels whose
// nodes have few chunks).
__global__ void __launch_bounds__(kBlock) k_select_last(uint32_t depth, uint32_t virt, uint32_t nsets,
                                                        const uint64_t* pre, const SetDesc* sets,
                                                        const DevParams* params, NodeSel* sel0,
                                                        uint32_t* hist0, const uint32_t* rows0,
                                                        uint32_t* cb0) {
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t total = pre[nsets];
  constexpr uint32_t wpb = kBlock / 64;
  for (uint64_t gn = (uint64_t)blockIdx.x * wpb + (threadIdx.x >> 6); gn < total;
       gn += (uint64_t)gridDim.x * wpb) {
    LastSel L;
    if (!last_sel_node(depth, virt, nsets, pre, sets, params, sel0, gn, &L)) continue;
    const SetDesc& S = *L.S;
    const uint64_t j = L.j, chunks = L.chunks;
    uint32_t* hist = hist0 + S.hist_off + (j << 8);
    const uint32_t* rows = rows0 + S.rows_off + j * chunks * kRowStride;
    uint32_t* chunk_base = cb_level(S, depth, cb0) + j * chunks * 2;
    uint32_t b, jeq;
    if (!last_digit_of(hist, 1u << L.w, L.rank, &b, &jeq)) {
      if (lane == 0) check_failed(L.P, kChkLastDigit);
      continue;
    }
    if (lane == 0) {
      NodeSel ns;
      ns.prefix = L.prefix;
      ns.rank = L.rank;
      ns.v = (L.prefix << L.w) | b;
      ns.jeq = jeq;
      sel_level(S, depth, sel0)[j] = ns;
    }
    // per-chunk counts of members below v (lt) and equal to v (eq), then an
    // exclusive scan over the node's chunks in rounds of 64 (chunk = round *
    // 64 + lane), four rounds of loads in flight
    uint32_t run_l = 0, run_e = 0;
    for (uint64_t r0 = 0; r0 < chunks; r0 += 4 * 64) {
      uint32_t lt[4], eq[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint64_t ch = r0 + (uint64_t)u * 64 + lane;
        lt[u] = eq[u] = 0;
        if (ch < chunks) {
          const uint32_t* row = rows + ch * kRowStride;
          const uint32_t lo = row[b], hi = row[b + 1];
          lt[u] = row[257] + lo;
          eq[u] = hi - lo;
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint64_t ch = r0 + (uint64_t)u * 64 + lane;
        const uint32_t il = wave_incl(lt[u]), ie = wave_incl(eq[u]);
        if (ch < chunks) {
          chunk_base[ch * 2 + 0] = run_l + il - lt[u];
          chunk_base[ch * 2 + 1] = run_e + ie - eq[u];
        }
        run_l += (uint32_t)__builtin_amdgcn_readlane((int)il, 63);
        run_e += (uint32_t)__builtin_amdgcn_readlane((int)ie, 63);
      }
    }
  }
}

// As k_select_last for levels whose nodes have many chunks (the top levels
// of a large set): one block per node, the chunk scan spread over the block
// (16 consecutive chunks per thread, all their loads in flight).
__global__ void __launch_bounds__(kBlock) k_select_last_wide(uint32_t depth, uint32_t virt, uint32_t nsets,
                                                             const uint64_t* pre,
                                                             const SetDesc* sets,
                                                             const DevParams* params,
                                                             NodeSel* sel0, uint32_t* hist0,
                                                             const uint32_t* rows0,
                                                             uint32_t* cb0) {
  constexpr uint32_t kPer = 16;
  __shared__ uint32_t bx[2];
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t total = pre[nsets];
  for (uint64_t gn = blockIdx.x; gn < total; gn += gridDim.x) {
    LastSel L;
    // every thread reads the set's status; a status set meanwhile by another
    // block must not split the block at the barriers below
    const bool mine = last_sel_node(depth, virt, nsets, pre, sets, params, sel0, gn, &L);
    if (!__syncthreads_and(mine ? 1 : 0)) continue;
    const SetDesc& S = *L.S;
    const uint64_t j = L.j, chunks = L.chunks;
    if (threadIdx.x < 64) {
      uint32_t b = 0, jeq = 0;
      const bool ok = last_digit_of(hist0 + S.hist_off + (j << 8), 1u << L.w, L.rank, &b, &jeq);
      if (lane == 0) {
        if (ok) {
          NodeSel ns;
          ns.prefix = L.prefix;
          ns.rank = L.rank;
          ns.v = (L.prefix << L.w) | b;
          ns.jeq = jeq;
          sel_level(S, depth, sel0)[j] = ns;
        } else {
          check_failed(L.P, kChkLastDigitWide);
        }
        bx[0] = ok ? 1u : 0u;
        bx[1] = b;
      }
    }
    __syncthreads();
    const bool ok = bx[0] != 0;
    const uint32_t b = bx[1];
    __syncthreads();  // bx is rewritten by the next node
    if (!ok) continue;
    const uint32_t* rows = rows0 + S.rows_off + j * chunks * kRowStride;
    uint32_t* chunk_base = cb_level(S, depth, cb0) + j * chunks * 2;
    uint64_t run = 0;  // (lt << 32) | eq before this round
    for (uint64_t r0 = 0; r0 < chunks; r0 += (uint64_t)kPer * kBlock) {
      const uint64_t c0 = r0 + (uint64_t)threadIdx.x * kPer;
      uint32_t lt[kPer], eq[kPer];
      uint64_t mine = 0;
#pragma unroll
      for (uint32_t u = 0; u < kPer; ++u) {
        lt[u] = eq[u] = 0;
        if (c0 + u < chunks) {
          const uint32_t* row = rows + (c0 + u) * kRowStride;
          const uint32_t lo = row[b], hi = row[b + 1];
          lt[u] = row[257] + lo;
          eq[u] = hi - lo;
        }
      }
#pragma unroll
      for (uint32_t u = 0; u < kPer; ++u) mine += ((uint64_t)lt[u] << 32) | eq[u];
      uint64_t tot;
      uint64_t at = run + block_exscan_u64(mine, &tot);
#pragma unroll
      for (uint32_t u = 0; u < kPer; ++u) {
        if (c0 + u < chunks) {
          chunk_base[(c0 + u) * 2 + 0] = (uint32_t)(at >> 32);
          chunk_base[(c0 + u) * 2 + 1] = (uint32_t)at;
        }
        at += ((uint64_t)lt[u] << 32) | eq[u];
      }
      run += tot;
    }
  }
}

// The next level's first-digit bins while a chunk is partitioned: kLhCopies
// copies per child (lane mod kLhCopies picks one), each 257 words apart so
// that equal bins of different copies sit in different LDS banks; few bins
// (32 for 13-bit codes) are hit by many lanes at once, and one copy made the
// atomics collide.
constexpr uint32_t kLhCopies = 4, kLhStride = 257;
constexpr uint32_t kLhWords = 2 * kLhCopies * kLhStride;
__device__ __forceinline__ uint32_t lh_slot(bool left, uint32_t bin) {
  return ((left ? 0u : kLhCopies) + (threadIdx.x & (kLhCopies - 1))) * kLhStride + bin;
}

// Stable partition of a chunk in streaming groups of kGroup elements:
// wavefront w of the block takes the 512 consecutive elements
// [g + 512 w, g + 512 w + 512) of a group as 8 rows of 64.  Codes are handled
// in axis order (split axis, next axis, third axis), so the split code is
// always k0 and the next level's code k1: no per-element axis selection.
// Ranks below / equal to the median come from ballots within the wavefront, a
// running count across its rows, and one exchange of wavefront totals per
// group (double-buffered: one barrier per group).  The next group's codes are
// loaded before that barrier, so they are in flight while this group waits
// and stores.
// With TRACK the source indices (when the set carries them) are loaded with
// the codes, so they are in flight together.
template <typename KT, bool FULL, bool TRACK>
__device__ __forceinline__ void scatter_load(uint32_t g, uint32_t end, const KT* A0, const KT* A1,
                                             const KT* A2, const uint32_t* is,
                                             uint32_t (&k)[3][kRows],
                                             uint32_t (&ki)[TRACK ? kRows : 1]) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wv = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const uint32_t base = g + wv * (kGroup / (kBlock / 64));
  const KT* a0 = A0 + base + lane;  // one 64-bit address per axis; rows are immediate offsets
  const KT* a1 = A1 + base + lane;
  const KT* a2 = A2 + base + lane;
#pragma unroll
  for (int i = 0; i < kRows; ++i) {
    const bool act = FULL || base + 64u * i + lane < end;
    k[0][i] = act ? (uint32_t)a0[64 * i] : 0u;
    k[1][i] = act ? (uint32_t)a1[64 * i] : 0u;
    k[2][i] = act ? (uint32_t)a2[64 * i] : 0u;
    if (TRACK) ki[i] = (act && is) ? is[base + 64u * i + lane] : 0u;
  }
}

template <bool FULL>
__device__ __forceinline__ void scatter_ranks(uint32_t g, uint32_t end, const uint32_t (&k)[3][kRows],
                                              uint32_t v, uint32_t (&rr)[kRows], uint32_t& wl,
                                              uint32_t& we) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wv = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const uint32_t base = g + wv * (kGroup / (kBlock / 64));
  wl = 0;
  we = 0;
#pragma unroll
  for (int i = 0; i < kRows; ++i) {
    const bool act = FULL || base + 64u * i + lane < end;
    const uint64_t mlt = __ballot(act && k[0][i] < v);
    const uint64_t meq = __ballot(act && k[0][i] == v);
    // ranks within the wavefront's 512 elements: below v | equal to v << 16
    rr[i] = (wl + lanes_below(mlt)) | ((we + lanes_below(meq)) << 16);
    wl += popc64(mlt);
    we += popc64(meq);
  }
}

template <typename KT, int NA, bool FULL, bool TRACK>
__device__ __forceinline__ void scatter_store(uint32_t g, uint32_t end, const uint32_t (&k)[3][kRows],
                                              const uint32_t (&ki)[TRACK ? kRows : 1],
                                              const uint32_t (&rr)[kRows], uint32_t bl,
                                              uint32_t be, KT* B0, KT* B1, KT* B2,
                                              const uint32_t* is, uint32_t* id, uint32_t sz,
                                              uint32_t v, uint32_t jeq, bool cl, bool cr,
                                              uint32_t shn, uint32_t maskn, uint32_t* lhist,
                                              DevParams* P) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wv = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const uint32_t base = g + wv * (kGroup / (kBlock / 64));
  const uint32_t half = sz >> 1;
#pragma unroll
  for (int i = 0; i < kRows; ++i) {
    const uint32_t p = base + 64u * i + lane;
    if (!FULL && p >= end) continue;
    const bool lt = k[0][i] < v, eq = k[0][i] == v;
    const uint32_t L = bl + (rr[i] & 0xffffu), E = be + (rr[i] >> 16);
    const uint32_t lb = L + umin32(E, jeq);
    const bool left = lt || (eq && E < jeq);
    const uint32_t dest = left ? lb : half + (p - lb);
    if (dest < sz) {
      B0[dest] = (KT)k[0][i];
      if (NA > 1) B1[dest] = (KT)k[1][i];
      if (NA > 2) B2[dest] = (KT)k[2][i];
      if (TRACK && is)
        id[dest] = ki[i];
      else if (!TRACK && is)
        id[dest] = is[p];
      if (left ? cl : cr)
        atomicAdd(&lhist[lh_slot(left, (NA > 1 ? k[1][i] : k[0][i]) >> shn & maskn)], 1u);
    } else {
      check_failed(P, kChkScatterStore);
    }
  }
}

// Staged variant of scatter_store: each element goes to its slot in the
// group's output order in LDS (stg: three axes of kGroup words, then the
// source indices), left-goers first.  The group's left-goers land in one
// contiguous run of the node and its right-goers in another, so the drain
// below writes both runs with consecutive lanes on consecutive slots (stores
// straight from the ranks interleave the two runs within every instruction).
template <int NA, bool FULL, bool TRACK>
__device__ __forceinline__ void scatter_stage(uint32_t g, uint32_t end, const uint32_t (&k)[3][kRows],
                                              const uint32_t (&ki)[TRACK ? kRows : 1],
                                              const uint32_t (&rr)[kRows], uint32_t bl,
                                              uint32_t be, uint32_t lbg, uint32_t nl,
                                              uint32_t v, uint32_t jeq, bool cl, bool cr,
                                              uint32_t shn, uint32_t maskn, uint32_t* lhist,
                                              uint32_t* stg, bool track, DevParams* P) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wv = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const uint32_t base = g + wv * (kGroup / (kBlock / 64));
#pragma unroll
  for (int i = 0; i < kRows; ++i) {
    const uint32_t p = base + 64u * i + lane;
    if (!FULL && p >= end) continue;
    const bool lt = k[0][i] < v, eq = k[0][i] == v;
    const uint32_t L = bl + (rr[i] & 0xffffu), E = be + (rr[i] >> 16);
    const uint32_t lb = L + umin32(E, jeq);
    const bool left = lt || (eq && E < jeq);
    const uint32_t loc = left ? lb - lbg : nl + (p - g) - (lb - lbg);
    if (loc < (uint32_t)kGroup) {
      stg[loc] = k[0][i];
      if (NA > 1) stg[kGroup + loc] = k[1][i];
      if (NA > 2) stg[2 * kGroup + loc] = k[2][i];
      if (TRACK) stg[3 * kGroup + loc] = ki[i];  // (zero when the set carries none)
      if (left ? cl : cr)
        atomicAdd(&lhist[lh_slot(left, (NA > 1 ? k[1][i] : k[0][i]) >> shn & maskn)], 1u);
    } else {
      check_failed(P, kChkScatterStage);
    }
  }
}

// Writes a staged group: output t < nl is the left-goer at node slot lbg + t,
// the others the right-goers from slot half + (g - lbg) on.
template <typename KT, int NA, bool TRACK>
__device__ __forceinline__ void scatter_drain(uint32_t g, uint32_t gsz, uint32_t lbg, uint32_t nl,
                                              uint32_t half, uint32_t sz, KT* B0, KT* B1, KT* B2,
                                              uint32_t* id, const uint32_t* stg, DevParams* P) {
  const uint32_t rbase = half + (g - lbg) - nl;
#pragma unroll
  for (int i = 0; i < kRows; ++i) {
    const uint32_t t = threadIdx.x + (uint32_t)kBlock * i;
    if (t >= gsz) break;
    const uint32_t dest = t < nl ? lbg + t : rbase + t;
    if (dest < sz) {
      B0[dest] = (KT)stg[t];
      if (NA > 1) B1[dest] = (KT)stg[kGroup + t];
      if (NA > 2) B2[dest] = (KT)stg[2 * kGroup + t];
      if (TRACK && id) id[dest] = stg[3 * kGroup + t];
    } else {
      check_failed(P, kChkScatterDrain);
    }
  }
}

template <typename KT, int NA, bool TRACK, bool STAGE>
__device__ __forceinline__ void scatter_range(uint32_t beg, uint32_t end, const KT* A0, const KT* A1, const KT* A2,
                              KT* B0, KT* B1, KT* B2, const uint32_t* is, uint32_t* id,
                              uint32_t sz, uint32_t v, uint32_t jeq, uint32_t lt_run,
                              uint32_t eq_run, bool cl, bool cr, uint32_t shn, uint32_t maskn,
                              uint32_t* lhist, uint32_t* stg, DevParams* P) {
  __shared__ __align__(16) uint32_t cnt[2][kBlock / 64][2];
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wv = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  uint32_t k[3][kRows], kn[3][kRows];
  uint32_t ki[TRACK ? kRows : 1], kin[TRACK ? kRows : 1];
  if (beg >= end) return;
  if (beg + kGroup <= end)
    scatter_load<KT, true, TRACK>(beg, end, A0, A1, A2, is, k, ki);
  else
    scatter_load<KT, false, TRACK>(beg, end, A0, A1, A2, is, k, ki);
  int buf = 0;
  for (uint32_t g = beg; g < end; g += kGroup, buf ^= 1) {
    const bool full = g + kGroup <= end;
    uint32_t rr[kRows], wl, we;
    if (full)
      scatter_ranks<true>(g, end, k, v, rr, wl, we);
    else
      scatter_ranks<false>(g, end, k, v, rr, wl, we);
    const uint32_t gn = g + kGroup;
    if (gn < end) {
      if (gn + kGroup <= end)
        scatter_load<KT, true, TRACK>(gn, end, A0, A1, A2, is, kn, kin);
      else
        scatter_load<KT, false, TRACK>(gn, end, A0, A1, A2, is, kn, kin);
    }
    if (lane == 0) cnt[buf][wv][0] = wl, cnt[buf][wv][1] = we;
    __syncthreads();
    const uint4 X = *(const uint4*)&cnt[buf][0][0];  // wavefronts 0, 1
    const uint4 Y = *(const uint4*)&cnt[buf][2][0];  // wavefronts 2, 3
    const uint32_t bl = lt_run + (wv > 0 ? X.x : 0u) + (wv > 1 ? X.z : 0u) + (wv > 2 ? Y.x : 0u);
    const uint32_t be = eq_run + (wv > 0 ? X.y : 0u) + (wv > 1 ? X.w : 0u) + (wv > 2 ? Y.y : 0u);
    const uint32_t lbg = lt_run + umin32(eq_run, jeq);  // left-goers before the group
    lt_run += X.x + X.z + Y.x + Y.z;
    eq_run += X.y + X.w + Y.y + Y.w;
    if (STAGE) {
      // the previous group's drain finished before the barrier above
      const uint32_t nl = lt_run + umin32(eq_run, jeq) - lbg;
      if (full)
        scatter_stage<NA, true, TRACK>(g, end, k, ki, rr, bl, be, lbg, nl, v, jeq, cl, cr, shn,
                                       maskn, lhist, stg, is != nullptr, P);
      else
        scatter_stage<NA, false, TRACK>(g, end, k, ki, rr, bl, be, lbg, nl, v, jeq, cl, cr, shn,
                                        maskn, lhist, stg, is != nullptr, P);
      __syncthreads();
      scatter_drain<KT, NA, TRACK>(g, full ? (uint32_t)kGroup : end - g, lbg, nl, sz >> 1, sz, B0, B1,
                                   B2, id, stg, P);
    } else if (full) {
      scatter_store<KT, NA, true, TRACK>(g, end, k, ki, rr, bl, be, B0, B1, B2, is, id, sz, v,
                                         jeq, cl, cr, shn, maskn, lhist, P);
    } else {
      scatter_store<KT, NA, false, TRACK>(g, end, k, ki, rr, bl, be, B0, B1, B2, is, id, sz, v,
                                          jeq, cl, cr, shn, maskn, lhist, P);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int i = 0; i < kRows; ++i) k[a][i] = kn[a][i];
    if (TRACK)
#pragma unroll
      for (int i = 0; i < kRows; ++i) ki[i] = kin[i];
  }
}

template <typename KT, bool TRACK, bool STAGE>
__device__ void scatter_body(uint32_t depth, const SetDesc& S, DevParams* P, const LevelCtx& c,
                             uint32_t v, uint32_t jeq, uint32_t lt_run, uint32_t eq_run,
                             const uint8_t* src, uint8_t* dst, const uint32_t* isrc, uint32_t* idst,
                             uint32_t* hist, uint32_t* lhist, uint32_t* stg) {
  static_assert(kBlock == 256, "four wavefronts per block");
  const uint64_t n = S.n, kst = S.kst;
  const uint32_t dims = S.dims, r = S.r;
  const uint32_t d = depth % dims;
  const uint64_t j = c.lb / c.sh.chunks, ch = c.lb % c.sh.chunks;
  uint64_t st, sz64;
  node_span(n, depth, j, &st, &sz64);
  const uint64_t beg64 = ch * (uint64_t)c.sh.chunk_elems;
  if (beg64 >= sz64) return;
  // positions inside the node fit 32 bits (n < 2^32)
  const uint32_t sz = (uint32_t)sz64, beg = (uint32_t)beg64;
  const uint32_t end = (uint32_t)(beg64 + c.sh.chunk_elems < sz64 ? beg64 + c.sh.chunk_elems : sz64);
  const uint32_t* is = isrc ? isrc + st : nullptr;
  uint32_t* id = idst ? idst + st : nullptr;
  if (STAGE && !TRACK && is) {  // the staged path carries indices only with TRACK
    if (threadIdx.x == 0) check_failed(P, kChkStageIdx);
    return;
  }
  if (sz <= r) {  // leaf: copy through
    const KT* s0 = (const KT*)src + st;
    KT* d0 = (KT*)dst + st;
    for (uint32_t p = beg + threadIdx.x; p < end; p += blockDim.x) {
      d0[p] = s0[p];
      if (dims > 1) d0[kst + p] = s0[kst + p];
      if (dims > 2) d0[2 * kst + p] = s0[2 * kst + p];
      if (is) id[p] = is[p];
    }
    return;
  }
  // next level's first digit, built here when that level runs a mid pass
  const uint32_t half = sz >> 1;
  const uint32_t dn = (depth + 1) % dims;
  const DigitPlan pn = digit_plan(P->G[dn]);
  // (not for wavefront levels, whose medians work on registers or on codes
  // minus the node minimum)
  const bool fuse = depth + 1 < S.gl && pn.npass >= 2 && level_kind(n, depth + 1) != kLevelWave &&
                    !level_fused(S, depth + 1);
  const uint32_t wn = pn.width[0], shn = pn.shift[0], maskn = (1u << wn) - 1;
  const bool cl = fuse && half > r, cr = fuse && (sz - half) > r;  // children that split again
  if (fuse)
    for (uint32_t i = threadIdx.x; i < kLhWords; i += kBlock) lhist[i] = 0;
  // axis order: split axis, next axis, third axis
  const uint32_t a1 = dims > 1 ? dn : d, a2 = dims > 2 ? (d + 2) % dims : d;
  const KT* A0 = (const KT*)src + st + (uint64_t)d * kst;
  const KT* A1 = (const KT*)src + st + (uint64_t)a1 * kst;
  const KT* A2 = (const KT*)src + st + (uint64_t)a2 * kst;
  KT* B0 = (KT*)dst + st + (uint64_t)d * kst;
  KT* B1 = (KT*)dst + st + (uint64_t)a1 * kst;
  KT* B2 = (KT*)dst + st + (uint64_t)a2 * kst;
  if (dims == 3)
    scatter_range<KT, 3, TRACK, STAGE>(beg, end, A0, A1, A2, B0, B1, B2, is, id, sz, v, jeq, lt_run,
                                       eq_run, cl, cr, shn, maskn, lhist, stg, P);
  else  // fewer axes: the missing ones repeat the split axis (same value, same slot)
    scatter_range<KT, 3, TRACK, STAGE>(beg, end, A0, A1, A0, B0, B1, B0, is, id, sz, v, jeq, lt_run,
                                       eq_run, cl, cr, shn, maskn, lhist, stg, P);
  if (fuse) {
    __syncthreads();
    for (uint32_t child = 0; child < 2; ++child) {
      uint32_t cnum = 0;
#pragma unroll
      for (uint32_t cp = 0; cp < kLhCopies; ++cp)
        cnum += lhist[(child * kLhCopies + cp) * kLhStride + threadIdx.x];
      if (cnum) atomicAdd(&hist_level(S, depth + 1, hist)[((2 * j + child) << 8) + threadIdx.x], cnum);
    }
  }
}

// TRACK: some set of the batch carries source indices (loaded with the codes).
// STAGE: groups are staged in LDS before the stores (levels whose chunks hold
// many groups; with one or two groups per block the extra barrier and LDS
// round trip cost more than the coalesced stores save).
template <bool TRACK, bool STAGE>
__global__ void __launch_bounds__(kBlock) k_scatter(uint32_t depth, uint32_t nsets,
                                                    const uint64_t* pre, const SetDesc* sets,
                                                    DevParams* params, const NodeSel* sel0,
                                                    const uint32_t* cb0, uint8_t* src0,
                                                    uint8_t* dst0, uint32_t* isrc0,
                                                    uint32_t* idst0, uint32_t* hist0) {
  const LevelCtx c = level_ctx(nsets, pre, sets, depth);
  const SetDesc& S = sets[c.s];
  DevParams* P = params + c.s;
  if (P->status != BBX_OK) return;
  if (level_is_local(S.n, depth) || pair_first(S, depth) || pair_second(S, depth)) return;
  __shared__ uint32_t lhist[kLhWords];
  __shared__ uint32_t stg[STAGE ? (TRACK ? 4 : 3) * kGroup : 1];  // one staged group (codes, indices)
  level_bufs(S, depth, src0, dst0, isrc0, idst0);
  const uint32_t* isrc = S.track ? isrc0 + S.idx_off : nullptr;
  uint32_t* idst = S.track ? idst0 + S.idx_off : nullptr;
  const NodeSel ns = sel_level(S, depth, sel0)[c.lb / c.sh.chunks];
  const uint32_t* cb = cb_level(S, depth, cb0) + c.lb * 2;
  if (P->key16)
    scatter_body<uint16_t, TRACK, STAGE>(depth, S, P, c, ns.v, ns.jeq, cb[0], cb[1], src0 + S.key_off,
                                        dst0 + S.key_off, isrc, idst, hist0 + S.hist_off, lhist, stg);
  else
    scatter_body<uint32_t, TRACK, STAGE>(depth, S, P, c, ns.v, ns.jeq, cb[0], cb[1], src0 + S.key_off,
                                        dst0 + S.key_off, isrc, idst, hist0 + S.hist_off, lhist, stg);
}

// Median of one node's axis codes, inside one block: radix passes of at most
// 8 bits, either over the code's own digits with the first digit's bins
// already counted by the partition above (`hist`), or over the codes minus
// the node minimum after a pass for the node's code range (the re-reads of a
// node of at most a few hundred KB mostly hit the cache).  Returns the median
// code v and how many members equal to v precede it (they go left).
template <typename KT>
__device__ void local_median(const KT* axis, uint64_t A, uint64_t B, uint32_t rank, uint32_t* v_out,
                             uint32_t* jeq_out, uint32_t* bins, uint32_t* red, uint32_t* hist,
                             const DigitPlan& pl) {
  const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // with `hist` the digits are those of the code itself (the set's digit
  // plan) and the first one's bins are already counted there; else they are
  // digits of the code minus the node minimum, widest first
  uint32_t mn = 0, Gs = pl.shift[0] + pl.width[0];
  if (!hist) {
    uint32_t lo = 0xffffffffu, hi = 0;
    scan_codes(axis, A, B, [&](uint32_t q) {
      lo = q < lo ? q : lo;
      hi = q > hi ? q : hi;
    });
    for (int o = 32; o > 0; o >>= 1) {
      const uint32_t a = __shfl_xor(lo, o), b = __shfl_xor(hi, o);
      lo = a < lo ? a : lo;
      hi = b > hi ? b : hi;
    }
    if (lane == 0) red[wv] = lo, red[4 + wv] = hi;
    __syncthreads();
    mn = red[0] < red[1] ? (red[0] < red[2] ? (red[0] < red[3] ? red[0] : red[3])
                                            : (red[2] < red[3] ? red[2] : red[3]))
                         : (red[1] < red[2] ? (red[1] < red[3] ? red[1] : red[3])
                                            : (red[2] < red[3] ? red[2] : red[3]));
    uint32_t mx = red[4];
    for (int k = 5; k < 8; ++k) mx = red[k] > mx ? red[k] : mx;
    Gs = bitlen32(mx - mn);
  }
  uint32_t prefix = 0, used = 0;
  // the first pass sees every member, so it spreads them over up to 256
  // bins; later passes see only the members that match the prefix found so
  // far
  for (uint32_t pass = 0; used < Gs; ++pass) {
    const uint32_t w = hist ? dp_width(pl, pass) : (Gs - used < 8 ? Gs - used : 8);
    const uint32_t hs = Gs - used;
    used += w;
    const uint32_t sh = Gs - used, mask = (1u << w) - 1;
    if (hist && pass == 0) {
      bins[threadIdx.x] = hist[threadIdx.x];
      hist[threadIdx.x] = 0;  // zero again for the next use of these bins
      __syncthreads();
    } else {
      bins[threadIdx.x] = 0;
      __syncthreads();
      scan_codes(axis, A, B, [&](uint32_t q) {
        const uint32_t k = q - mn;
        if ((k >> hs) == prefix) atomicAdd(&bins[(k >> sh) & mask], 1u);
      });
      __syncthreads();
    }
    if (wv == 0) {  // one wavefront finds the bin holding the rank
      uint32_t c[4], mine = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) c[k] = bins[lane * 4 + k], mine += c[k];
      uint32_t cum = wave_incl(mine) - mine;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (cum <= rank && rank < cum + c[k]) red[8] = lane * 4 + k, red[9] = rank - cum;
        cum += c[k];
      }
    }
    __syncthreads();
    prefix = (prefix << w) | red[8];
    rank = red[9];
    __syncthreads();  // red and bins are rewritten by the next pass
  }
  *v_out = mn + prefix;
  *jeq_out = rank;
}

// A level whose nodes each fit one block: median and stable partition of
// each node in one block, for every set whose level is local.
__global__ void __launch_bounds__(kBlock) k_level_local(uint32_t depth, uint32_t nsets,
                                                        const uint64_t* pre, const SetDesc* sets,
                                                        DevParams* params, uint8_t* src0,
                                                        uint8_t* dst0, uint32_t* isrc0,
                                                        uint32_t* idst0, uint32_t* hist0) {
  const LevelCtx c = level_ctx(nsets, pre, sets, depth);
  const SetDesc& S = sets[c.s];
  DevParams* P = params + c.s;
  if (P->status != BBX_OK) return;
  if (level_kind(S.n, depth) != kLevelBlock || level_fused(S, depth)) return;
  __shared__ uint32_t lhist[kLhWords];
  __shared__ uint32_t red[16];
  level_bufs(S, depth, src0, dst0, isrc0, idst0);
  const uint32_t* isrc = S.track ? isrc0 + S.idx_off : nullptr;
  uint32_t* idst = S.track ? idst0 + S.idx_off : nullptr;
  uint64_t st, sz;
  node_span(S.n, depth, c.lb, &st, &sz);
  uint32_t v = 0, jeq = 0;
  const uint32_t d = depth % S.dims;
  const uint8_t* keys = src0 + S.key_off;
  if (sz > S.r) {
    const DigitPlan pl = digit_plan(P->G[d]);
    // the level above built this node's first-digit histogram when the code
    // has more than one digit (depth 0 has none for a block-local level)
    uint32_t* h = depth > 0 && pl.npass >= 2
                      ? hist_level(S, depth, hist0 + S.hist_off) + (c.lb << 8) : nullptr;
    if (P->key16)
      local_median((const uint16_t*)keys + (uint64_t)d * S.kst, st, st + sz, (uint32_t)(sz >> 1), &v,
                   &jeq, lhist, red, h, pl);
    else
      local_median((const uint32_t*)keys + (uint64_t)d * S.kst, st, st + sz, (uint32_t)(sz >> 1), &v,
                   &jeq, lhist, red, h, pl);
    __syncthreads();  // lhist is reused by the partition
  }
  if (P->key16)
    scatter_body<uint16_t, false, false>(depth, S, P, c, v, jeq, 0, 0, src0 + S.key_off,
                                         dst0 + S.key_off, isrc, idst, hist0 + S.hist_off, lhist,
                                         nullptr);
  else
    scatter_body<uint32_t, false, false>(depth, S, P, c, v, jeq, 0, 0, src0 + S.key_off,
                                         dst0 + S.key_off, isrc, idst, hist0 + S.hist_off, lhist,
                                         nullptr);
}

// Median of a node's axis codes by one wavefront (nodes of at most kWaveNode
// members): code range by DPP reductions, then radix passes of at most 8 bits
// (widest first) over codes minus the minimum, in the wavefront's own bins.
template <typename KT>
__device__ void wave_median(const KT* axis, uint32_t sz, uint32_t rank, uint32_t* bins,
                            uint32_t* v_out, uint32_t* jeq_out) {
  const uint32_t lane = threadIdx.x & 63;
  const KT* al = axis + lane;
  uint32_t lo = 0xffffffffu, hi = 0;
  for (uint32_t b = 0; b < sz; b += 512) {  // 8 loads in flight per lane
    uint32_t q[8];
    if (b + 512 <= sz) {
#pragma unroll
      for (int u = 0; u < 8; ++u) q[u] = (uint32_t)al[b + 64 * u];
#pragma unroll
      for (int u = 0; u < 8; ++u) lo = umin32(lo, q[u]), hi = umax32(hi, q[u]);
    } else {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const uint32_t e = b + 64 * u + lane;
        q[u] = e < sz ? (uint32_t)axis[e] : 0xffffffffu;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (b + 64 * u + lane < sz) {
          lo = umin32(lo, q[u]);
          hi = umax32(hi, q[u]);
        }
      }
    }
  }
  const uint32_t mn = wave_min_dpp(lo);
  const uint32_t Gs = bitlen32(wave_max_dpp(hi) - mn);
  uint32_t prefix = 0, used = 0;
  while (used < Gs) {
    const uint32_t w = Gs - used < 8 ? Gs - used : 8;
    const uint32_t hs = Gs - used;
    used += w;
    const uint32_t sh = Gs - used, mask = (1u << w) - 1;
#pragma unroll
    for (int k = 0; k < 4; ++k) bins[lane * 4 + k] = 0;
    wave_sync();
    for (uint32_t b = 0; b < sz; b += 512) {
      uint32_t q[8];
      const bool full = b + 512 <= sz;
      if (full) {
#pragma unroll
        for (int u = 0; u < 8; ++u) q[u] = (uint32_t)al[b + 64 * u];
      } else {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const uint32_t e = b + 64 * u + lane;
          q[u] = e < sz ? (uint32_t)axis[e] : 0u;
        }
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const uint32_t k = q[u] - mn;
        if ((full || b + 64 * u + lane < sz) && (k >> hs) == prefix)
          atomicAdd(&bins[(k >> sh) & mask], 1u);
      }
    }
    wave_sync();
    uint32_t c[4], mine = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) c[k] = bins[lane * 4 + k], mine += c[k];
    uint32_t cum = wave_incl(mine) - mine;
    uint32_t fb = 0, fr = 0;
    bool found = false;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (cum <= rank && rank < cum + c[k]) found = true, fb = lane * 4 + k, fr = rank - cum;
      cum += c[k];
    }
    const uint64_t fm = __ballot(found);
    const int fl = fm ? __ffsll((unsigned long long)fm) - 1 : 0;
    prefix = (prefix << w) | (uint32_t)__builtin_amdgcn_readlane((int)fb, fl);
    rank = (uint32_t)__builtin_amdgcn_readlane((int)fr, fl);
    wave_sync();  // the bins are cleared by the next pass
  }
  *v_out = mn + prefix;
  *jeq_out = rank;
}

// 512 members of a node by one wavefront (8 rows of 64), codes in axis order
// (split axis first); ballots give each member's rank among the members
// below / equal to the median before it.
template <typename KT, bool FULL, bool TRACK>
__device__ __forceinline__ void wave_part_rows(uint32_t base, uint32_t sz, const KT* A0,
                                               const KT* A1, const KT* A2, KT* B0, KT* B1, KT* B2,
                                               const uint32_t* is, uint32_t* id, uint32_t v,
                                               uint32_t jeq, uint32_t& lt_run, uint32_t& eq_run,
                                               DevParams* P) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t half = sz >> 1;
  uint32_t k0[8], k1[8], k2[8], ix[TRACK ? 8 : 1];
  {
    const KT* a0 = A0 + base + lane;
    const KT* a1 = A1 + base + lane;
    const KT* a2 = A2 + base + lane;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const bool act = FULL || base + 64u * i + lane < sz;
      k0[i] = act ? (uint32_t)a0[64 * i] : 0u;
      k1[i] = act ? (uint32_t)a1[64 * i] : 0u;
      k2[i] = act ? (uint32_t)a2[64 * i] : 0u;
      if (TRACK) ix[i] = (act && is) ? is[base + 64u * i + lane] : 0u;  // with the codes
    }
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const uint32_t p = base + 64u * i + lane;
    const bool act = FULL || p < sz;
    const bool lt = k0[i] < v, eq = k0[i] == v;
    const uint64_t mlt = __ballot(act && lt), meq = __ballot(act && eq);
    if (act) {
      const uint32_t L = lt_run + lanes_below(mlt);
      const uint32_t E = eq_run + lanes_below(meq);
      const uint32_t lb = L + umin32(E, jeq);
      const bool left = lt || (eq && E < jeq);
      const uint32_t dest = left ? lb : half + (p - lb);
      if (dest < sz) {
        B0[dest] = (KT)k0[i];
        B1[dest] = (KT)k1[i];
        B2[dest] = (KT)k2[i];
        if (TRACK && is)
          id[dest] = ix[i];
        else if (!TRACK && is)
          id[dest] = is[p];
      } else {
        check_failed(P, kChkWavePart);
      }
    }
    lt_run += (uint32_t)__popcll(mlt);
    eq_run += (uint32_t)__popcll(meq);
  }
}

// Stable partition of one node by one wavefront.  With fewer than three axes
// the missing ones repeat the split axis (the same value to the same slot).
template <typename KT, bool TRACK>
__device__ void wave_partition(const KT* src, KT* dst, uint64_t kst, const uint32_t* is,
                               uint32_t* id, uint32_t dims, uint32_t d, uint32_t sz, uint32_t v,
                               uint32_t jeq, DevParams* P) {
  const uint32_t a1 = dims > 1 ? (d + 1) % dims : d, a2 = dims > 2 ? (d + 2) % dims : d;
  const KT* A0 = src + (uint64_t)d * kst;
  const KT* A1 = src + (uint64_t)a1 * kst;
  const KT* A2 = src + (uint64_t)a2 * kst;
  KT* B0 = dst + (uint64_t)d * kst;
  KT* B1 = dst + (uint64_t)a1 * kst;
  KT* B2 = dst + (uint64_t)a2 * kst;
  uint32_t lt_run = 0, eq_run = 0;
  for (uint32_t base = 0; base < sz; base += 512) {
    if (base + 512 <= sz)
      wave_part_rows<KT, true, TRACK>(base, sz, A0, A1, A2, B0, B1, B2, is, id, v, jeq, lt_run,
                                      eq_run, P);
    else
      wave_part_rows<KT, false, TRACK>(base, sz, A0, A1, A2, B0, B1, B2, is, id, v, jeq, lt_run,
                                       eq_run, P);
  }
}

template <typename KT, bool TRACK>
__device__ void level_wave_body(uint32_t depth, const SetDesc& S, DevParams* P, uint64_t j,
                                const uint8_t* src, uint8_t* dst, const uint32_t* isrc,
                                uint32_t* idst, uint32_t* bins) {
  uint64_t st, sz64;
  node_span(S.n, depth, j, &st, &sz64);
  const uint32_t sz = (uint32_t)sz64;
  const uint32_t dims = S.dims, d = depth % dims;
  const uint64_t kst = S.kst;
  const KT* s0 = (const KT*)src + st;
  KT* d0 = (KT*)dst + st;
  const uint32_t* is = isrc ? isrc + st : nullptr;
  uint32_t* id = idst ? idst + st : nullptr;
  if (level_fused(S, depth)) return;  // levels of k_level_fused
  if (sz <= S.r) {  // leaf: copy through
    for (uint32_t p = threadIdx.x & 63; p < sz; p += 64) {
      d0[p] = s0[p];
      if (dims > 1) d0[kst + p] = s0[kst + p];
      if (dims > 2) d0[2 * kst + p] = s0[2 * kst + p];
      if (is) id[p] = is[p];
    }
    return;
  }
  uint32_t v, jeq;
  wave_median(s0 + (uint64_t)d * kst, sz, sz >> 1, bins, &v, &jeq);
  wave_partition<KT, TRACK>(s0, d0, kst, is, id, dims, d, sz, v, jeq, P);
}

// Levels whose nodes have at most kWaveNode members: one wavefront per node,
// four nodes per block, no block barriers.
template <bool TRACK>
__global__ void __launch_bounds__(kBlock) k_level_wave(uint32_t depth, uint32_t nsets,
                                                       const uint64_t* pre, const SetDesc* sets,
                                                       DevParams* params, uint8_t* src0,
                                                       uint8_t* dst0, uint32_t* isrc0,
                                                       uint32_t* idst0) {
  __shared__ uint32_t bins[kBlock / 64][256];
  const uint32_t wv = threadIdx.x >> 6;
  const uint64_t gn = (uint64_t)blockIdx.x * (kBlock / 64) + wv;
  if (gn >= pre[nsets]) return;  // whole wavefront
  const uint32_t s = find_set(pre, nsets, gn);
  const SetDesc& S = sets[s];
  DevParams* P = params + s;
  if (P->status != BBX_OK) return;
  if (level_kind(S.n, depth) != kLevelWave) return;
  const uint64_t j = gn - pre[s];
  level_bufs(S, depth, src0, dst0, isrc0, idst0);
  const uint32_t* isrc = S.track ? isrc0 + S.idx_off : nullptr;
  uint32_t* idst = S.track ? idst0 + S.idx_off : nullptr;
  if (P->key16)
    level_wave_body<uint16_t, TRACK>(depth, S, P, j, src0 + S.key_off, dst0 + S.key_off, isrc, idst,
                                     bins[wv]);
  else
    level_wave_body<uint32_t, TRACK>(depth, S, P, j, src0 + S.key_off, dst0 + S.key_off, isrc, idst,
                                     bins[wv]);
}

// ---------------------------------------------------------------- fused levels

// Pairs of levels run as one in-place pass with a node's codes in registers:
// W wavefronts per node (1: nodes of at most kFuseNode members, four nodes
// per block; 4: nodes of at most 4 kFuseNode, one node per block), each
// wavefront holding R = kFuseNode / 64 rows of 64 consecutive members
// (wavefront w: members [w kFuseNode, (w + 1) kFuseNode)).
constexpr int kFuseRows = (int)(kFuseNode / 64);

// sum over the wavefront (uniform result)
__device__ inline uint32_t wave_sum(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_readlane((int)wave_incl(x), 63);
}

template <int W>
__device__ inline void fuse_sync() {
  if (W == 1)
    wave_sync();
  else
    __syncthreads();
}

// Per-wavefront totals t[0..K) (uniform within each wavefront) -> the sum
// over the node's lower wavefronts (member order is wavefront-major).  Each
// exchange of a node has an xs array of its own (nothing is reused).
template <int W, int K>
__device__ inline void fuse_bases(const uint32_t (&t)[K], uint32_t (&b)[K], uint32_t (*xs)[4]) {
  static_assert(K <= 4, "four totals per exchange");
#pragma unroll
  for (int k = 0; k < K; ++k) b[k] = 0;
  if (W == 1) return;
  const uint32_t wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) xs[wv][k] = t[k];
  __syncthreads();
#pragma unroll
  for (int w = 0; w < W; ++w)
#pragma unroll
    for (int k = 0; k < K; ++k) b[k] += (uint32_t)w < wv ? xs[w][k] : 0u;
}

// Radix select over the node's codes held in registers, for one or two
// member groups at once: group g's member of rank rank[g] among the members
// flagged in the lanes' bit masks m[g] (bit i: the lane's i-th member),
// ordered by (code, member order).  Widest digit first, at most 8 bits per
// pass, over the code range of all flagged members; pass p counts group g
// into bins [512 (p & 1) + 256 g, ... + 256) and the scanning wavefront
// posts its finds in red[2 W + 4 (p & 1) ...], so that a pass needs no
// barrier after its reads: the next pass uses the other half, and the one
// after it comes after the next pass's barriers.  Returns each group's code
// in v[g] and, in rank[g], how many members equal to it precede it.  The
// bins are zero on entry and on return (the scanning wavefront clears what
// it read); red[0, 2 W) (the code range) is rewritten only after a later
// barrier of the caller.
template <int R, int W, int NG, typename Q>
__device__ void reg_select(const Q& q, const uint32_t (&m)[NG], uint32_t (&rank)[NG],
                           uint32_t* bins, uint32_t* red, uint32_t (&v)[NG]) {
  static_assert(NG == 1 || NG == 2, "one or two groups");
  const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint32_t all = NG == 1 ? m[0] : (m[0] | m[NG - 1]);
  uint32_t lo, hi;
  q.minmax(all, &lo, &hi);
  uint32_t mn = wave_min_dpp(lo), mx = wave_max_dpp(hi);
  if (W > 1) {
    if (lane == 0) red[wv] = mn, red[W + wv] = mx;
    __syncthreads();
    mn = red[0], mx = red[W];
#pragma unroll
    for (int w = 1; w < W; ++w) mn = umin32(mn, red[w]), mx = umax32(mx, red[W + w]);
  }
  const uint32_t Gs = mx > mn ? bitlen32(mx - mn) : 0u;
  uint32_t prefix[NG];
#pragma unroll
  for (int g = 0; g < NG; ++g) prefix[g] = 0;
  uint32_t used = 0, half = 0;
  while (used < Gs) {
    const uint32_t w = Gs - used < 8 ? Gs - used : 8;
    const uint32_t hs = Gs - used;
    used += w;
    uint32_t* const bn = bins + 512 * half;
    uint32_t* const rd = red + 2 * W + 4 * half;
    half ^= 1;
    const uint32_t sh = Gs - used, mask = (1u << w) - 1;
    if (hs == Gs) {  // first pass: every flagged member is a candidate
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const uint32_t k = q[i] - mn;
        const uint32_t g0 = NG == 2 && ((m[NG - 1] >> i) & 1u) ? 256u : 0u;
        if ((all >> i) & 1u) atomicAdd(&bn[g0 + ((k >> sh) & mask)], 1u);
      }
    } else {
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const uint32_t k = q[i] - mn;
        const bool g1 = NG == 2 && ((m[NG - 1] >> i) & 1u);
        const uint32_t pre = g1 ? prefix[NG - 1] : prefix[0];
        if (((all >> i) & 1u) && (k >> hs) == pre)
          atomicAdd(&bn[(g1 ? 256u : 0u) + ((k >> sh) & mask)], 1u);
      }
    }
    fuse_sync<W>();
    if (W == 1 || wv == 0) {  // the node's (first) wavefront finds the bin of each rank
      uint32_t c[NG][4], mine = 0;
#pragma unroll
      for (int g = 0; g < NG; ++g)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          c[g][k] = bn[256 * g + lane * 4 + k];
          mine += c[g][k] << (16 * g);  // a group's counts stay below 2^16
        }
#pragma unroll
      for (int g = 0; g < NG; ++g)
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (c[g][k]) bn[256 * g + lane * 4 + k] = 0;
      const uint32_t cum = wave_incl(mine) - mine;
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        uint32_t cg = (cum >> (16 * g)) & 0xffffu, fb = 0, fr = 0;
        bool found = false;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          if (cg <= rank[g] && rank[g] < cg + c[g][k]) found = true, fb = lane * 4 + k, fr = rank[g] - cg;
          cg += c[g][k];
        }
        const uint64_t fm = __ballot(found);
        const int fl = fm ? __ffsll((unsigned long long)fm) - 1 : 0;
        fb = (uint32_t)__builtin_amdgcn_readlane((int)fb, fl);
        fr = (uint32_t)__builtin_amdgcn_readlane((int)fr, fl);
        if (W == 1) {
          prefix[g] = (prefix[g] << w) | fb;
          rank[g] = fr;
        } else if (lane == 0) {
          rd[2 * g] = fb, rd[2 * g + 1] = fr;
        }
      }
    }
    if (W > 1) {
      __syncthreads();
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        prefix[g] = (prefix[g] << w) | rd[2 * g];
        rank[g] = rd[2 * g + 1];
      }
    }
  }
#pragma unroll
  for (int g = 0; g < NG; ++g) v[g] = mn + prefix[g];
}

// exclusive prefix over the wavefront; the wavefront total in *tot
__device__ inline uint32_t wave_excl(uint32_t x, uint32_t* tot) {
  const uint32_t incl = wave_incl(x);
  *tot = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
  return incl - x;
}

// R consecutive elements [p0, p0 + R) of one array (those below s; fill
// beyond) held by a lane, loaded with 16-byte loads when the array is
// 16-byte aligned and the run is whole; 16-bit codes two to a register.
template <typename T, int R>
struct RegRun {
  static constexpr int V = 16 / sizeof(T), PER = 4 / sizeof(T);
  static_assert(R % V == 0, "whole vectors");
  uint32_t w[R / PER];
  __device__ __forceinline__ uint32_t operator[](int i) const {
    return PER == 1 ? w[i] : ((i & 1) ? w[i >> 1] >> 16 : w[i >> 1] & 0xffffu);
  }
  // smallest and largest of the elements flagged in m (bit i: element i);
  // 16-bit codes of a lane whose every element is flagged go two at a time
  __device__ __forceinline__ void minmax(uint32_t m, uint32_t* lo, uint32_t* hi) const {
    uint32_t a = 0xffffffffu, b = 0;
    if (PER == 2 && m == (1u << R) - 1u) {
      typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
      u16x2 a2 = {0xffff, 0xffff}, b2 = {0, 0};
#pragma unroll
      for (int k = 0; k < R / PER; ++k) {
        const u16x2 x = __builtin_bit_cast(u16x2, w[k]);
        a2 = __builtin_elementwise_min(a2, x);
        b2 = __builtin_elementwise_max(b2, x);
      }
      a = umin32(a2.x, a2.y);
      b = umax32(b2.x, b2.y);
    } else {
#pragma unroll
      for (int i = 0; i < R; ++i)
        if ((m >> i) & 1u) a = umin32(a, (*this)[i]), b = umax32(b, (*this)[i]);
    }
    *lo = a;
    *hi = b;
  }
  __device__ __forceinline__ void load(const T* X, uint32_t p0, uint32_t s, bool vec, T fill) {
    if (vec && p0 + R <= s) {
#pragma unroll
      for (int b = 0; b < R / V; ++b) {
        const uint4 u = *(const uint4*)(X + p0 + b * V);
        w[4 * b + 0] = u.x, w[4 * b + 1] = u.y, w[4 * b + 2] = u.z, w[4 * b + 3] = u.w;
      }
    } else {
#pragma unroll
      for (int k = 0; k < R / PER; ++k) {
        uint32_t x = 0;
#pragma unroll
        for (int h = 0; h < PER; ++h) {
          const uint32_t p = p0 + (uint32_t)(k * PER + h);
          x |= (uint32_t)(p < s ? X[p] : fill) << (16 * h);
        }
        w[k] = x;
      }
    }
  }
};

// Stores E consecutive values [e0, e0 + E) (those below s) to X, with
// 16-byte stores when X is 16-byte aligned and the run is whole; get(k)
// gives the value of slot e0 + k.
template <int E, typename T, typename F>
__device__ inline void store_run(T* X, uint32_t e0, uint32_t s, bool vec, F&& get) {
  constexpr int V = 16 / sizeof(T);
  static_assert(E % V == 0, "whole vectors");
  if (vec && e0 + E <= s) {
#pragma unroll
    for (int b = 0; b < E / V; ++b) {
      union {
        uint4 u;
        T e[V];
      } x;
#pragma unroll
      for (int k = 0; k < V; ++k) x.e[k] = (T)get((uint32_t)(b * V + k));
      *(uint4*)(X + e0 + b * V) = x.u;
    }
  } else {
#pragma unroll
    for (int k = 0; k < E; ++k)
      if (e0 + k < s) X[e0 + k] = (T)get((uint32_t)k);
  }
}

// Marks v as rewritten (no instruction), so that values derived from it
// before this point are not kept live past it but derived again after it.
template <typename T>
__device__ __forceinline__ void reg_fence(T& v) {
  asm volatile("" : "+v"(v));
}
template <typename T, int R>
__device__ __forceinline__ void reg_fence(RegRun<T, R>& q) {
#pragma unroll
  for (int k = 0; k < R * (int)sizeof(T) / 4; ++k) reg_fence(q.w[k]);
}

// Levels k and k + 1 of one node, in place.  Each lane holds R consecutive
// members (member order: wavefront, lane, row) with their codes (and source
// indices) in registers.  The node's median along d is selected there, then
// both children's medians along the next axis in one joint select.  Every
// member's side, its side in its child and finally its slot come from
// per-lane counts and one wavefront scan per phase (ties go left in member
// order), and the node is permuted through LDS and written back with
// coalesced stores.  Equal to two stable partitions: the children keep the
// node's member order, and the grandchildren the children's.  Each array of
// the node is read before the barrier that precedes the first store to it
// (a value is consumed before the barrier, so its load has returned), and no
// other wavefront or block touches the node.  `lds` holds the select bins,
// then the staged node (three 16-bit arrays with 16-bit codes, else one
// 32-bit array at a time).  Every lane holds R members: those past the
// node's end read as the top code of their axis, so they order after every
// member of the node (a code as large or larger, a later member) and leave
// each median, side and slot of the node's members as it is; they all fall
// in the last grandchild, at slots s and up, which are never written back.
template <typename KT, bool TRACK, int W>
__device__ __forceinline__ void level_fused_body(uint32_t depth, const SetDesc& S, DevParams* P,
                                                 uint64_t j, uint8_t* keys, uint32_t* idx,
                                                 uint32_t* lds, uint32_t* red, uint32_t (*xs)[W][4]) {
  constexpr int R = kFuseRows;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wv = W == 1 ? 0u : (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  uint64_t st, sz64;
  node_span(S.n, depth, j, &st, &sz64);
  if (sz64 > (uint64_t)W * kFuseNode || sz64 <= S.r) {  // launch plan violated: never expected
    if (threadIdx.x == 0) check_failed(P, kChkFusedIdx);
    return;
  }
  const uint32_t s = (uint32_t)sz64;
  const uint32_t dims = S.dims, d = depth % dims;
  const uint32_t a1 = (d + 1) % dims, a2 = dims > 2 ? (d + 2) % dims : d;
  const uint64_t kst = S.kst;
  KT* X0 = (KT*)keys + st + (uint64_t)d * kst;
  KT* X1 = (KT*)keys + st + (uint64_t)a1 * kst;
  KT* X2 = (KT*)keys + st + (uint64_t)a2 * kst;
  uint32_t* I = idx ? idx + st : nullptr;
  // the code arrays are 64-element aligned per axis, so one test covers all
  const bool vk = (st % (16 / sizeof(KT))) == 0, vi = (st % 4) == 0;
  const uint32_t p0 = wv * (uint32_t)kFuseNode + lane * R;  // the lane's first member
  RegRun<KT, R> q0, q1;  // the split axis and the next one (the third axis, and
                         // the source indices, are read when they are staged)
  auto top = [](uint32_t g) { return (KT)(g >= 32 ? 0xffffffffu : (1u << g) - 1u); };
  q0.load(X0, p0, s, vk, top(P->G[d]));
  q1.load(X1, p0, s, vk, top(P->G[a1]));
  constexpr uint32_t all = (1u << R) - 1u;  // member flags: every member of the lane
  // between phases: the codes are taken up again from their packed
  // registers instead of holding unpacked copies across the phases
  auto fence = [&]() { reg_fence(q0), reg_fence(q1); };
  for (uint32_t k = W == 1 ? lane : threadIdx.x; k < 1024; k += 64u * W) lds[k] = 0;  // select bins
  // every load of the node has returned before any wavefront of the node
  // passes its first barrier (the stores come after it)
  __builtin_amdgcn_s_waitcnt(0);
  fuse_sync<W>();

  // ---- level k: the node's median along d; each member's side (members
  // equal to the median go left while fewer than jeq of them did)
  uint32_t v, jeq;
  {
    const uint32_t m1[1] = {all};
    uint32_t rk[1] = {s >> 1}, vv[1];
    reg_select<R, W, 1>(q0, m1, rk, lds, red, vv);
    v = vv[0], jeq = rk[0];
  }
  fence();
  uint32_t ne = 0;
#pragma unroll
  for (int i = 0; i < R; ++i) ne += q0[i] == v ? 1u : 0u;
  uint32_t te[1], be[1];
  uint32_t erun = wave_excl(ne, &te[0]);
  fuse_bases<W, 1>(te, be, xs[0]);
  erun += be[0];
  uint32_t left = 0;
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const bool eq = q0[i] == v;
    if (q0[i] < v || (eq && erun < jeq)) left |= 1u << i;
    erun += eq ? 1u : 0u;
  }
  const uint32_t right = all & ~left;
  fence();

  // ---- level k + 1: both children's medians along the next axis, then each
  // member's side within its child (counts of the two children packed in
  // the 16-bit halves of one word: they stay below 2^16)
  const uint32_t sL = s >> 1, sR = s - sL, hL = sL >> 1, hR = sR >> 1;
  uint32_t vL, vR, jL, jR;
  {
    const uint32_t m2[2] = {left, right};
    uint32_t rk[2] = {hL, hR}, vv[2];
    reg_select<R, W, 2>(q1, m2, rk, lds, red, vv);
    vL = vv[0], vR = vv[1], jL = rk[0], jR = rk[1];
  }
  fence();
  uint32_t ne2 = 0;
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const bool l = (left >> i) & 1u;
    if (q1[i] == (l ? vL : vR)) ne2 += l ? 1u : 0x10000u;
  }
  uint32_t t2, b2[2];
  uint32_t run2 = wave_excl(ne2, &t2);
  {
    const uint32_t tt[2] = {t2 & 0xffffu, t2 >> 16};
    fuse_bases<W, 2>(tt, b2, xs[1]);
  }
  run2 += b2[0] | (b2[1] << 16);
  // grandchild of each member: g = 0 LL [0, hL), 1 LR [hL, sL), 2 RL
  // [sL, sL + hR), 3 RR [sL + hR, s), two bits per member in gm
  uint32_t gm = 0;
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const bool l = (left >> i) & 1u;
    const uint32_t vs = l ? vL : vR, js = l ? jL : jR;
    const uint32_t run = l ? (run2 & 0xffffu) : (run2 >> 16);
    const bool eq = q1[i] == vs;
    const bool f = q1[i] < vs || (eq && run < js);
    gm |= ((l ? 0u : 2u) | (f ? 0u : 1u)) << (2 * i);
    run2 += eq ? (l ? 1u : 0x10000u) : 0u;
  }

  // ---- slots: a lane's member counts per grandchild, 16 bits apiece in one
  // 64-bit word (they stay below 2^16), one scan per 32-bit half; c holds
  // each grandchild's next slot
  fence();
  uint64_t cnt = 0;
#pragma unroll
  for (int i = 0; i < R; ++i) cnt += 1ull << (16 * ((gm >> (2 * i)) & 3u));
  uint32_t tA, tB, b4[4];
  const uint32_t rA = wave_excl((uint32_t)cnt, &tA), rB = wave_excl((uint32_t)(cnt >> 32), &tB);
  {
    const uint32_t tt[4] = {tA & 0xffffu, tA >> 16, tB & 0xffffu, tB >> 16};
    fuse_bases<W, 4>(tt, b4, xs[2]);
  }
  // C member slots: every grandchild must count its own size (the last also
  // the members past the node's end), then each member's slot lies inside
  // its grandchild (the last wavefront sees the node totals)
  constexpr uint32_t C = W * kFuseNode;
  if (wv == W - 1) {
    const uint32_t tt[4] = {tA & 0xffffu, tA >> 16, tB & 0xffffu, tB >> 16};
    const uint32_t gs[4] = {hL, sL - hL, hR, sR - hR + (C - s)};
    bool bad = false;
#pragma unroll
    for (int g = 0; g < 4; ++g) bad |= b4[g] + tt[g] != gs[g];
    if (bad && lane == 0) check_failed(P, kChkFusedPart);
  }
  uint64_t c = ((uint64_t)rB << 32 | rA) +
               ((uint64_t)b4[0] | ((uint64_t)(hL + b4[1]) << 16) | ((uint64_t)(sL + b4[2]) << 32) |
                ((uint64_t)(sL + hR + b4[3]) << 48));
  // the mask keeps even a failed count's slots inside LDS
  uint32_t dst[R];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const uint32_t sh = 16 * ((gm >> (2 * i)) & 3u);
    dst[i] = (uint32_t)(c >> sh) & (C - 1);
    c += 1ull << sh;
  }
  // ---- the node permuted through LDS, then written back in slot order with
  // 8 consecutive slots per thread and round
  constexpr uint32_t T = 64u * W, E = 8;
  const uint32_t tid = W == 1 ? lane : threadIdx.x;
  if constexpr (sizeof(KT) == 2) {
    RegRun<KT, R> q2;
    q2.load(X2, p0, s, vk, 0);  // no store to the node before the barrier below
    // one array of C 16-bit slots per axis, copied out 16 bytes at a time
    uint16_t* sg = (uint16_t*)lds;
#pragma unroll
    for (int i = 0; i < R; ++i) {
      sg[dst[i]] = (uint16_t)q0[i];
      sg[C + dst[i]] = (uint16_t)q1[i];
      if (dims > 2) sg[2 * C + dst[i]] = (uint16_t)q2[i];
    }
    fuse_sync<W>();
    auto out = [&](KT* X, const uint16_t* g, uint32_t e0) {
      if (vk && e0 + E <= s) {
        *(uint4*)(X + e0) = *(const uint4*)(g + e0);
      } else {
#pragma unroll
        for (uint32_t k = 0; k < E; ++k)
          if (e0 + k < s) X[e0 + k] = g[e0 + k];
      }
    };
    for (uint32_t e0 = tid * E; e0 < s; e0 += T * E) {
      out(X0, sg, e0);
      out(X1, sg + C, e0);
      if (dims > 2) out(X2, sg + 2 * C, e0);
    }
  }
  // 32-bit codes and source indices: one array at a time, each read from
  // the node before any wavefront stores to it
  uint32_t* stg32 = lds;
  auto pass32 = [&](auto* X, const auto& val, bool vec) {
#pragma unroll
    for (int i = 0; i < R; ++i) stg32[dst[i]] = val[i];
    fuse_sync<W>();
    for (uint32_t e0 = tid * E; e0 < s; e0 += T * E)
      store_run<E>(X, e0, s, vec, [&](uint32_t k) { return stg32[e0 + k]; });
    fuse_sync<W>();  // the next array reuses the staging area
  };
  if constexpr (sizeof(KT) == 4) {
    fuse_sync<W>();
    pass32(X0, q0, vk);
    pass32(X1, q1, vk);
    if (dims > 2) {
      RegRun<KT, R> q2;
      q2.load(X2, p0, s, vk, 0);
      pass32(X2, q2, vk);
    }
  }
  if constexpr (TRACK) {
    if (I) {
      fuse_sync<W>();
      RegRun<uint32_t, R> ix;
      ix.load(I, p0, s, vi, 0);
      pass32(I, ix, vi);
    }
  }
}

// Levels k and k + 1 of the sets whose fused depth for W wavefronts per node
// is k.  W = 1: one wavefront per node of depth k, four nodes per block;
// W = 4 or 16: one block of W wavefronts per node.
template <int W>
constexpr int fused_threads() { return W == 1 ? kBlock : 64 * W; }
template <bool TRACK, int W>
__global__ void __launch_bounds__(fused_threads<W>(), W == 4 ? 4 : 1) k_level_fused(uint32_t depth, uint32_t nsets,
                                                        const uint64_t* pre, const SetDesc* sets,
                                                        DevParams* params, uint8_t* keys0,
                                                        uint8_t* keys1, uint32_t* idx0,
                                                        uint32_t* idx1) {
  static_assert(W == 1 || W == 4 || W == 16, "a wavefront or a block of 4 or 16 per node");
  // per node (W = 1: per wavefront) the select bins, then the staged node:
  // three 16-bit arrays of W kFuseNode members (3/4 of a u64 per member)
  constexpr uint32_t kNodeWords = 3 * W * (uint32_t)kFuseNode / 4;
  constexpr uint32_t kNodes = W == 1 ? kBlock / 64 : 1;
  __shared__ __align__(16) uint64_t stage[kNodes * kNodeWords];
  __shared__ uint32_t red[2 * W + 8];
  __shared__ uint32_t xs[3][W][4];
  const uint32_t wv = threadIdx.x >> 6;
  const uint64_t gn = W == 1 ? (uint64_t)blockIdx.x * (kBlock / 64) + wv : blockIdx.x;
  if (gn >= pre[nsets]) return;  // whole wavefront (W = 1) or block
  const uint32_t s = find_set(pre, nsets, gn);
  const SetDesc& S = sets[s];
  DevParams* P = params + s;
  if (P->status != BBX_OK) return;
  if ((W == 1 ? S.fuse_depth : W == 4 ? S.fuse_depth4 : S.fuse_depth16) != depth) return;
  const uint64_t j = gn - pre[s];
  level_bufs(S, depth, keys0, keys1, idx0, idx1);  // in place: the buffer holding the codes
  uint32_t* idx = S.track ? idx0 + S.idx_off : nullptr;
  uint32_t* b = (uint32_t*)(stage + (W == 1 ? wv * kNodeWords : 0));
  if (P->key16)
    level_fused_body<uint16_t, TRACK, W>(depth, S, P, j, keys0 + S.key_off, idx, b, red, xs);
  else
    level_fused_body<uint32_t, TRACK, W>(depth, S, P, j, keys0 + S.key_off, idx, b, red, xs);
}

// ---------------------------------------------------------------- paired levels
//
// Global levels k (even) and k + 1 of a set with npairs > k / 2 move the codes
// once.  After level k's selects (as for any global level):
//   k_label          per chunk of level k: each member's side (left / right
//                    child) as one bit, in the chunk's order, and the
//                    children's first-digit bins of the next axis
//   (selects)        level k + 1's radix select over its nodes, which still
//                    lie inside their parents: k_lab_hist for further digits
//                    and the last one (rows per child and parent chunk),
//                    k_select_mid / k_select_last with virt = 1
//   k_scatter4       per chunk of level k: both sides of every member, then
//                    one stable four-way partition to the grandchildren, and
//                    the first-digit bins of level k + 2
// Equal to the two stable partitions: the members of each child keep their
// order, those of each grandchild their child's order.

// The side labels of a chunk: one 64-bit word per row of 64 members, at
// (chunk's block) * chunk_elems / 64 + (row's first member - chunk start) / 64.
__device__ inline uint64_t* chunk_labels(const SetDesc& S, const LevelCtx& c, uint64_t* lab0) {
  return lab0 + S.lab_off + c.lb * (uint64_t)(c.sh.chunk_elems / 64);
}

// Level k's sides of one chunk, written as labels, and the children's
// first-digit bins of the next axis when that code has more than one digit.
template <typename KT>
__device__ void label_body(uint32_t depth, const SetDesc& S, DevParams* P, const LevelCtx& c,
                           uint32_t v, uint32_t jeq, uint32_t lt_run, uint32_t eq_run,
                           const uint8_t* src, uint64_t* lab, uint32_t* hist, uint32_t* lhist) {
  const uint64_t n = S.n;
  const uint32_t dims = S.dims, d = depth % dims, dn = (depth + 1) % dims;
  const uint64_t j = c.lb / c.sh.chunks, ch = c.lb % c.sh.chunks;
  uint64_t st, sz64;
  node_span(n, depth, j, &st, &sz64);
  const uint64_t beg64 = ch * (uint64_t)c.sh.chunk_elems;
  if (beg64 >= sz64) return;
  const uint32_t beg = (uint32_t)beg64;
  const uint32_t end = (uint32_t)(beg64 + c.sh.chunk_elems < sz64 ? beg64 + c.sh.chunk_elems : sz64);
  const DigitPlan pn = digit_plan(P->G[dn]);
  const bool fuse = pn.npass >= 2;  // both children split again (pairing asks for it)
  const uint32_t shn = pn.shift[0], maskn = (1u << pn.width[0]) - 1;
  if (fuse)
    for (uint32_t i = threadIdx.x; i < kLhWords; i += kBlock) lhist[i] = 0;
  const KT* A0 = (const KT*)src + st + (uint64_t)d * S.kst;
  const KT* A1 = (const KT*)src + st + (uint64_t)dn * S.kst;
  __shared__ __align__(16) uint32_t cnt[2][kBlock / 64][2];
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wv = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  int buf = 0;
  for (uint32_t g = beg; g < end; g += kGroup, buf ^= 1) {
    const uint32_t base = g + wv * (kGroup / (kBlock / 64));
    uint32_t k0[kRows], k1[kRows];
#pragma unroll
    for (int i = 0; i < kRows; ++i) {
      const uint32_t p = base + 64u * i + lane;
      k0[i] = p < end ? (uint32_t)A0[p] : 0u;
      k1[i] = p < end ? (uint32_t)A1[p] : 0u;
    }
    uint32_t rr[kRows], wl = 0, we = 0;
#pragma unroll
    for (int i = 0; i < kRows; ++i) {
      const bool act = base + 64u * i + lane < end;
      const uint64_t mlt = __ballot(act && k0[i] < v);
      const uint64_t meq = __ballot(act && k0[i] == v);
      rr[i] = lanes_below(meq);
      we += popc64(meq);
      wl += popc64(mlt);
    }
    if (lane == 0) cnt[buf][wv][0] = wl, cnt[buf][wv][1] = we;
    __syncthreads();
    const uint4 X = *(const uint4*)&cnt[buf][0][0];
    const uint4 Y = *(const uint4*)&cnt[buf][2][0];
    uint32_t be = eq_run + (wv > 0 ? X.y : 0u) + (wv > 1 ? X.w : 0u) + (wv > 2 ? Y.y : 0u);
    lt_run += X.x + X.z + Y.x + Y.z;
    eq_run += X.y + X.w + Y.y + Y.w;
#pragma unroll
    for (int i = 0; i < kRows; ++i) {
      const bool act = base + 64u * i + lane < end;
      const bool eq = k0[i] == v;
      const bool left = k0[i] < v || (eq && be + rr[i] < jeq);
      const uint64_t mr = __ballot(act && !left);
      be += popc64(__ballot(act && eq));
      if (lane == 0) lab[(base - beg) / 64 + i] = mr;
      if (fuse && act) atomicAdd(&lhist[lh_slot(left, (k1[i] >> shn) & maskn)], 1u);
    }
  }
  if (fuse) {
    __syncthreads();
    for (uint32_t child = 0; child < 2; ++child) {
      uint32_t cnum = 0;
#pragma unroll
      for (uint32_t cp = 0; cp < kLhCopies; ++cp)
        cnum += lhist[(child * kLhCopies + cp) * kLhStride + threadIdx.x];
      if (cnum) atomicAdd(&hist_level(S, depth + 1, hist)[((2 * j + child) << 8) + threadIdx.x], cnum);
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_label(uint32_t depth, uint32_t nsets,
                                                  const uint64_t* pre, const SetDesc* sets,
                                                  DevParams* params, const NodeSel* sel0,
                                                  const uint32_t* cb0, uint8_t* keys0,
                                                  uint8_t* keys1, uint64_t* lab0,
                                                  uint32_t* hist0) {
  const LevelCtx c = level_ctx(nsets, pre, sets, depth);
  const SetDesc& S = sets[c.s];
  DevParams* P = params + c.s;
  if (P->status != BBX_OK || !pair_first(S, depth)) return;
  __shared__ uint32_t lhist[kLhWords];
  const uint8_t* src = (key_buf(S, depth) ? keys1 : keys0) + S.key_off;
  const NodeSel ns = sel_level(S, depth, sel0)[c.lb / c.sh.chunks];
  const uint32_t* cb = cb_level(S, depth, cb0) + c.lb * 2;
  uint64_t* lab = chunk_labels(S, c, lab0);
  if (P->key16)
    label_body<uint16_t>(depth, S, P, c, ns.v, ns.jeq, cb[0], cb[1], src, lab, hist0 + S.hist_off, lhist);
  else
    label_body<uint32_t>(depth, S, P, c, ns.v, ns.jeq, cb[0], cb[1], src, lab, hist0 + S.hist_off, lhist);
}

// Level k + 1 (dv) of a pair, digit pass `pass` over one chunk of a level-k
// node: each member's child from its label, candidates matching the child's
// digits so far counted into the child's bins.  A mid pass adds the counts
// to the children's node bins; the last pass also writes each child's row
// for the chunk (prefix counts per bin, candidates, members below the
// digits so far), at rows (child * chunks + chunk).
template <typename KT, bool LAST>
__device__ void lab_hist_body(uint32_t dv, uint32_t pass, const SetDesc& S, const DevParams* P,
                              const LevelCtx& c, const uint8_t* src, const uint64_t* lab,
                              const NodeSel* sel, uint32_t* hist, uint32_t* rows0,
                              uint32_t* lh) {
  const uint64_t n = S.n;
  const uint32_t dn = dv % S.dims;
  const DigitPlan pl = digit_plan(P->G[dn]);
  const uint64_t j = c.lb / c.sh.chunks, ch = c.lb % c.sh.chunks;
  uint64_t st, sz64;
  node_span(n, dv - 1, j, &st, &sz64);
  const uint32_t w = dp_width(pl, pass), sh = dp_shift(pl, pass), hs = sh + w;
  const uint32_t pre0 = pass == 0 ? 0u : sel[2 * j].prefix;
  const uint32_t pre1 = pass == 0 ? 0u : sel[2 * j + 1].prefix;
  const uint32_t nb = 1u << w, mask = nb - 1;
  lh[threadIdx.x] = 0;
  lh[kBlock + threadIdx.x] = 0;
  __syncthreads();
  const uint64_t beg64 = ch * (uint64_t)c.sh.chunk_elems;
  const uint32_t beg = (uint32_t)(beg64 < sz64 ? beg64 : sz64);
  const uint32_t end = (uint32_t)(beg64 + c.sh.chunk_elems < sz64 ? beg64 + c.sh.chunk_elems : sz64);
  const KT* A1 = (const KT*)src + st + (uint64_t)dn * S.kst;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wv = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  uint32_t below0 = 0, below1 = 0;
  for (uint32_t g = beg; g < end; g += kGroup) {
    const uint32_t base = g + wv * (kGroup / (kBlock / 64));
    uint32_t k1[kRows];
    uint64_t lw[kRows];
#pragma unroll
    for (int i = 0; i < kRows; ++i) {
      const uint32_t p = base + 64u * i + lane;
      k1[i] = p < end ? (uint32_t)A1[p] : 0u;
      lw[i] = base + 64u * i < end ? lab[(base - beg) / 64 + i] : 0ull;
    }
#pragma unroll
    for (int i = 0; i < kRows; ++i) {
      const uint32_t p = base + 64u * i + lane;
      if (p >= end) continue;
      const bool right = (lw[i] >> lane) & 1u;
      const uint32_t hi = k1[i] >> hs, pre = right ? pre1 : pre0;
      if (LAST) {
        if (hi < pre) {
          if (right)
            ++below1;
          else
            ++below0;
        }
      }
      if (hi == pre) atomicAdd(&lh[(right ? kBlock : 0u) + ((k1[i] >> sh) & mask)], 1u);
    }
  }
  __syncthreads();
  for (uint32_t child = 0; child < 2; ++child) {
    const uint32_t cnt = threadIdx.x < nb ? lh[child * kBlock + threadIdx.x] : 0u;
    const uint64_t jc = 2 * j + child;
    if (LAST) {
      uint64_t tot;
      const uint64_t ex = block_exscan_u64(((uint64_t)(child ? below1 : below0) << 32) | cnt, &tot);
      uint32_t* row = rows0 + (jc * c.sh.chunks + ch) * kRowStride;
      row[threadIdx.x] = (uint32_t)ex;
      if (threadIdx.x == 0) {
        row[256] = (uint32_t)tot;
        row[257] = (uint32_t)(tot >> 32);
      }
    }
    if (threadIdx.x < nb && cnt) atomicAdd(&hist[(jc << 8) + threadIdx.x], cnt);
  }
}

// LAST = 0: a further digit pass (skipped by the sets that need none); 1: the last pass
template <bool LAST>
__global__ void __launch_bounds__(kBlock) k_lab_hist(uint32_t dv, uint32_t pass, uint32_t nsets,
                                                     const uint64_t* pre, const SetDesc* sets,
                                                     const DevParams* params, uint8_t* keys0,
                                                     uint8_t* keys1, const uint64_t* lab0,
                                                     const NodeSel* sel0, uint32_t* hist0,
                                                     uint32_t* rows0, const uint32_t* pass_need) {
  if (!LAST && !pass_need[dv * 4 + pass]) return;
  __shared__ uint32_t lh[2 * kBlock];
  const uint64_t total = pre[nsets];
  for (uint64_t vb = blockIdx.x; vb < total; vb += gridDim.x) {  // block-uniform
    const LevelCtx c = level_ctx(nsets, pre, sets, dv - 1, vb);
    const SetDesc& S = sets[c.s];
    const DevParams* P = params + c.s;
    if (P->status != BBX_OK || !pair_first(S, dv - 1)) continue;
    const uint32_t np = digit_plan(P->G[dv % S.dims]).npass;
    const uint32_t ps = LAST ? np - 1 : pass;
    if (!LAST && pass + 1 >= np) continue;
    const uint8_t* src = (key_buf(S, dv - 1) ? keys1 : keys0) + S.key_off;
    const uint64_t* lab = chunk_labels(S, c, (uint64_t*)lab0);
    if (P->key16)
      lab_hist_body<uint16_t, LAST>(dv, ps, S, P, c, src, lab, sel_level(S, dv, sel0),
                                    hist0 + S.hist_off, rows0 + S.rows_off, lh);
    else
      lab_hist_body<uint32_t, LAST>(dv, ps, S, P, c, src, lab, sel_level(S, dv, sel0),
                                    hist0 + S.hist_off, rows0 + S.rows_off, lh);
    __syncthreads();  // lh is reused by the next block's chunk
  }
}

// The four-way partition of one chunk of a level-k node.  Per group of
// kGroup members: level k's ranks (below / equal to v) and one exchange of
// wavefront counts give each member's side; the ranks of the members equal
// to their child's median, and a second exchange, give its side in the
// child; four ballots and a third exchange rank it among the members of
// its grandchild.  The group is staged in LDS as four runs (one per
// grandchild, each contiguous in the output) and written with coalesced
// stores.
constexpr uint32_t kLh4Copies = 2;
constexpr uint32_t kLh4Words = 4 * kLh4Copies * kLhStride;

template <typename KT, bool TRACK>
__device__ void scatter4_body(uint32_t depth, const SetDesc& S, DevParams* P, const LevelCtx& c,
                              const NodeSel* sel, const NodeSel* sel2, const uint32_t* cb,
                              const uint32_t* cb2, const uint8_t* src, uint8_t* dst,
                              const uint32_t* isrc, uint32_t* idst, uint32_t* hist,
                              uint32_t* lhist, uint32_t* stg) {
  static_assert(kBlock == 256, "four wavefronts per block");
  const uint64_t n = S.n, kst = S.kst;
  const uint32_t dims = S.dims, r = S.r;
  const uint32_t d = depth % dims, dn = (depth + 1) % dims, d2 = (depth + 2) % dims;
  const uint64_t j = c.lb / c.sh.chunks, ch = c.lb % c.sh.chunks;
  uint64_t st, sz64;
  node_span(n, depth, j, &st, &sz64);
  const uint64_t beg64 = ch * (uint64_t)c.sh.chunk_elems;
  if (beg64 >= sz64) return;
  const uint32_t sz = (uint32_t)sz64, beg = (uint32_t)beg64;
  const uint32_t end = (uint32_t)(beg64 + c.sh.chunk_elems < sz64 ? beg64 + c.sh.chunk_elems : sz64);
  // level k: median, ties that go left, counts before the chunk
  const uint32_t v = sel[j].v, jeq = sel[j].jeq;
  uint32_t lt_run = cb[0], eq_run = cb[1];
  // level k + 1: per child its median, ties that go left, and its members
  // below / equal to the median before the chunk (rows of child * chunks + chunk)
  uint32_t vc[2], jc[2], ltc[2], eqc[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    vc[q] = sel2[2 * j + q].v;
    jc[q] = sel2[2 * j + q].jeq;
    const uint32_t* b = cb2 + ((2 * j + q) * c.sh.chunks + ch) * 2;
    ltc[q] = b[0];
    eqc[q] = b[1];
  }
  const uint32_t sL = sz >> 1, sR = sz - sL, hL = sL >> 1, hR = sR >> 1;
  // each grandchild's next slot (node-relative): LL, LR, RL, RR
  const uint32_t nL = lt_run + umin32(eq_run, jeq), nR = beg - nL;
  const uint32_t a0 = ltc[0] + umin32(eqc[0], jc[0]), a1 = ltc[1] + umin32(eqc[1], jc[1]);
  uint32_t gb[4] = {a0, hL + (nL - a0), sL + a1, sL + hR + (nR - a1)};
  const uint32_t gsz4[4] = {hL, sL - hL, hR, sR - hR};
  // level k + 2's first-digit bins per grandchild (when it runs a mid pass)
  const DigitPlan p2 = digit_plan(P->G[d2]);
  const bool fuse = depth + 2 < S.gl && p2.npass >= 2 && level_kind(n, depth + 2) != kLevelWave &&
                    !level_fused(S, depth + 2);
  const uint32_t sh2 = p2.shift[0], mask2 = (1u << p2.width[0]) - 1;
  bool cg[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) cg[q] = fuse && gsz4[q] > r;
  if (fuse)
    for (uint32_t i = threadIdx.x; i < kLh4Words; i += kBlock) lhist[i] = 0;
  const KT* A0 = (const KT*)src + st + (uint64_t)d * kst;
  const KT* A1 = (const KT*)src + st + (uint64_t)dn * kst;
  const KT* A2 = (const KT*)src + st + (uint64_t)d2 * kst;
  KT* B0 = (KT*)dst + st + (uint64_t)d * kst;
  KT* B1 = (KT*)dst + st + (uint64_t)dn * kst;
  KT* B2 = (KT*)dst + st + (uint64_t)d2 * kst;
  const uint32_t* is = isrc ? isrc + st : nullptr;
  uint32_t* id = idst ? idst + st : nullptr;
  // one exchange array per phase: a phase's counts are read before the
  // barrier of the next phase, so each is free again by the next group
  __shared__ __align__(16) uint32_t x1[kBlock / 64][2];
  __shared__ uint32_t x2[kBlock / 64];
  __shared__ __align__(16) uint32_t x3[kBlock / 64][4];
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wv = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  uint32_t k[3][kRows], ki[TRACK ? kRows : 1];
  auto load = [&](uint32_t g, uint32_t (&kk)[3][kRows], uint32_t (&kki)[TRACK ? kRows : 1]) {
    const uint32_t base = g + wv * (kGroup / (kBlock / 64));
#pragma unroll
    for (int i = 0; i < kRows; ++i) {
      const uint32_t p = base + 64u * i + lane;
      const bool act = p < end;
      kk[0][i] = act ? (uint32_t)A0[p] : 0u;
      kk[1][i] = act ? (uint32_t)A1[p] : 0u;
      kk[2][i] = act ? (uint32_t)A2[p] : 0u;
      if (TRACK) kki[i] = (act && is) ? is[p] : 0u;
    }
  };
  load(beg, k, ki);
  for (uint32_t g = beg; g < end; g += kGroup) {
    const uint32_t base = g + wv * (kGroup / (kBlock / 64));
    const uint32_t gsz = end - g < (uint32_t)kGroup ? end - g : (uint32_t)kGroup;
    // ---- level k: ranks among the members equal to v
    uint32_t re[kRows], wl = 0, we = 0;
    uint64_t am[kRows];  // lanes holding a member, per row
#pragma unroll
    for (int i = 0; i < kRows; ++i) {
      const bool act = base + 64u * i + lane < end;
      am[i] = __ballot(act);
      const uint64_t mlt = __ballot(act && k[0][i] < v);
      const uint64_t meq = __ballot(act && k[0][i] == v);
      re[i] = we + lanes_below(meq);
      wl += popc64(mlt);
      we += popc64(meq);
    }
    // the next group's codes are in flight while this one is partitioned
    uint32_t kn[3][kRows], kin[TRACK ? kRows : 1];
    if (g + kGroup < end) load(g + kGroup, kn, kin);
    if (lane == 0) x1[wv][0] = wl, x1[wv][1] = we;
    __syncthreads();
    uint32_t be = eq_run;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
      be += (uint32_t)w < wv ? x1[w][1] : 0u;
      lt_run += x1[w][0];
      eq_run += x1[w][1];
    }
    // ---- level k + 1: each member's child, ranks among the child's members
    // equal to its median (both children packed in 16-bit halves)
    uint64_t rm[kRows];  // lanes whose member goes right at level k, per row
    uint32_t re2[kRows], w2 = 0;
#pragma unroll
    for (int i = 0; i < kRows; ++i) {
      const bool act = base + 64u * i + lane < end;
      const bool right = !(k[0][i] < v || (k[0][i] == v && be + re[i] < jeq));
      rm[i] = __ballot(act && right);
      const uint32_t vq = right ? vc[1] : vc[0];
      const uint64_t mq = __ballot(act && k[1][i] == vq);
      const uint64_t m0 = mq & ~rm[i], m1 = mq & rm[i];
      re2[i] = w2 + (lanes_below(m0) | (lanes_below(m1) << 16));
      w2 += popc64(m0) | (popc64(m1) << 16);
    }
    if (lane == 0) x2[wv] = w2;
    __syncthreads();
    uint32_t e0 = eqc[0], e1 = eqc[1];
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
      const uint32_t x = x2[w];
      if ((uint32_t)w < wv) e0 += x & 0xffffu, e1 += x >> 16;
      eqc[0] += x & 0xffffu;
      eqc[1] += x >> 16;
    }
    // ---- grandchild of each member (0 LL, 1 LR, 2 RL, 3 RR) and its rank
    // among the group's members of that grandchild: one ballot of the
    // second-level side, the four masks from it and the first-level side
    uint32_t gq = 0;  // two bits per row
    uint32_t r4[kRows];
    uint32_t c4[4] = {0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < kRows; ++i) {
      const bool right = (rm[i] >> lane) & 1u;
      const uint32_t vq = right ? vc[1] : vc[0], jq = right ? jc[1] : jc[0];
      const uint32_t eq2 = right ? e1 + (re2[i] >> 16) : e0 + (re2[i] & 0xffffu);
      const bool first = k[1][i] < vq || (k[1][i] == vq && eq2 < jq);
      const uint64_t ms = __ballot(!first) & am[i];  // second halves
      const uint64_t M[4] = {am[i] & ~rm[i] & ~ms, ~rm[i] & ms, rm[i] & ~ms, rm[i] & ms};
      const uint32_t q = (right ? 2u : 0u) | (first ? 0u : 1u);
      gq |= q << (2 * i);
      const uint64_t mine = q == 0 ? M[0] : q == 1 ? M[1] : q == 2 ? M[2] : M[3];
      r4[i] = (q == 0 ? c4[0] : q == 1 ? c4[1] : q == 2 ? c4[2] : c4[3]) + lanes_below(mine);
#pragma unroll
      for (int t = 0; t < 4; ++t) c4[t] += popc64(M[t]);
    }
    if (lane == 0) {
      x3[wv][0] = c4[0];
      x3[wv][1] = c4[1];
      x3[wv][2] = c4[2];
      x3[wv][3] = c4[3];
    }
    __syncthreads();
    // group totals per grandchild, this wavefront's base within them, and
    // the staging offset of each grandchild's run
    uint32_t tq[4] = {0, 0, 0, 0}, wb[4] = {0, 0, 0, 0};
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint32_t x = x3[w][q];
        if ((uint32_t)w < wv) wb[q] += x;
        tq[q] += x;
      }
    const uint32_t ro[4] = {0, tq[0], tq[0] + tq[1], tq[0] + tq[1] + tq[2]};
#pragma unroll
    for (int i = 0; i < kRows; ++i) {
      const uint32_t p = base + 64u * i + lane;
      if (p >= end) continue;
      const uint32_t q = (gq >> (2 * i)) & 3u;
      const uint32_t loc = (q == 0 ? ro[0] + wb[0] : q == 1 ? ro[1] + wb[1] : q == 2 ? ro[2] + wb[2]
                                                                                   : ro[3] + wb[3]) + r4[i];
      if (loc < (uint32_t)kGroup) {
        stg[loc] = k[0][i];
        stg[kGroup + loc] = k[1][i];
        stg[2 * kGroup + loc] = k[2][i];
        if (TRACK) stg[3 * kGroup + loc] = ki[i];
        if (q == 0 ? cg[0] : q == 1 ? cg[1] : q == 2 ? cg[2] : cg[3])
          atomicAdd(&lhist[(q * kLh4Copies + (threadIdx.x & (kLh4Copies - 1))) * kLhStride +
                           ((k[2][i] >> sh2) & mask2)], 1u);
      } else {
        check_failed(P, kChkPairStage);
      }
    }
    __syncthreads();
    // drain: output t of the group belongs to run q when ro[q] <= t < ro[q + 1]
    // (the next group stages only after its first barrier, when this drain
    // is done)
#pragma unroll
    for (int i = 0; i < kRows; ++i) {
      const uint32_t t = threadIdx.x + (uint32_t)kBlock * i;
      if (t >= gsz) break;
      const uint32_t q = t >= ro[3] ? 3u : t >= ro[2] ? 2u : t >= ro[1] ? 1u : 0u;
      const uint32_t dest = (q == 0 ? gb[0] : q == 1 ? gb[1] : q == 2 ? gb[2] : gb[3]) + t -
                            (q == 0 ? 0u : q == 1 ? ro[1] : q == 2 ? ro[2] : ro[3]);
      if (dest < sz) {
        B0[dest] = (KT)stg[t];
        B1[dest] = (KT)stg[kGroup + t];
        if (dims > 2) B2[dest] = (KT)stg[2 * kGroup + t];
        if (TRACK && id) id[dest] = stg[3 * kGroup + t];
      } else {
        check_failed(P, kChkPairStore);
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) gb[q] += tq[q];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int i = 0; i < kRows; ++i) k[a][i] = kn[a][i];
    if (TRACK)
#pragma unroll
      for (int i = 0; i < kRows; ++i) ki[i] = kin[i];
  }
  __syncthreads();  // every wavefront's bins are counted
  if (fuse) {
    for (uint32_t q = 0; q < 4; ++q) {
      uint32_t cnum = 0;
#pragma unroll
      for (uint32_t cp = 0; cp < kLh4Copies; ++cp)
        cnum += lhist[(q * kLh4Copies + cp) * kLhStride + threadIdx.x];
      if (cnum) atomicAdd(&hist_level(S, depth + 2, hist)[((4 * j + q) << 8) + threadIdx.x], cnum);
    }
  }
}

template <bool TRACK>
__global__ void __launch_bounds__(kBlock) k_scatter4(uint32_t depth, uint32_t nsets,
                                                     const uint64_t* pre, const SetDesc* sets,
                                                     DevParams* params, const NodeSel* sel0,
                                                     const uint32_t* cb0, uint8_t* src0,
                                                     uint8_t* dst0, uint32_t* isrc0,
                                                     uint32_t* idst0, uint32_t* hist0) {
  const LevelCtx c = level_ctx(nsets, pre, sets, depth);
  const SetDesc& S = sets[c.s];
  DevParams* P = params + c.s;
  if (P->status != BBX_OK || !pair_first(S, depth)) return;
  __shared__ uint32_t lhist[kLh4Words];
  __shared__ uint32_t stg[(TRACK ? 4 : 3) * kGroup];
  level_bufs(S, depth, src0, dst0, isrc0, idst0);
  const uint32_t* isrc = S.track ? isrc0 + S.idx_off : nullptr;
  uint32_t* idst = S.track ? idst0 + S.idx_off : nullptr;
  if (!TRACK && isrc) {  // the launch carries indices for every set that has them
    if (threadIdx.x == 0) check_failed(P, kChkStageIdx);
    return;
  }
  const NodeSel* sel = sel_level(S, depth, sel0);
  const NodeSel* sel2 = sel_level(S, depth + 1, sel0);
  const uint32_t* cb = cb_level(S, depth, cb0) + c.lb * 2;
  const uint32_t* cb2 = cb_level(S, depth + 1, cb0);
  if (P->key16)
    scatter4_body<uint16_t, TRACK>(depth, S, P, c, sel, sel2, cb, cb2, src0 + S.key_off,
                                   dst0 + S.key_off, isrc, idst, hist0 + S.hist_off, lhist, stg);
  else
    scatter4_body<uint32_t, TRACK>(depth, S, P, c, sel, sel2, cb, cb2, src0 + S.key_off,
                                   dst0 + S.key_off, isrc, idst, hist0 + S.hist_off, lhist, stg);
}

// blocks of a select launch: one wavefront per node up to 8192 blocks, then striding
static uint64_t sel_grid(uint64_t nodes) {
  const uint64_t b = (nodes + kBlock / 64 - 1) / (kBlock / 64);
  return b < 8192 ? (b ? b : 1) : 8192;
}

// Levels k and k + 1 of the paired sets, after level k's selects.
hipError_t launch_pair(const BatchPlan& bp, const Ws& w, uint32_t k, hipStream_t s) {
  const uint64_t* plv = w.pre + bp.o_lv[k];
  const uint64_t* pnd2 = w.pre + bp.o_nd[k + 1];
  uint8_t* K0 = w.keys[0];
  uint8_t* K1 = w.keys[1];
  BBX_LAUNCH("pair_label", k_label, bp.g_lv[k], kBlock, 0, s, k, bp.nsets, plv, w.sets, w.params,
             w.sel, w.chunk_base, K0, K1, w.labels, w.hist);
  for (uint32_t pass = 0; pass < 3; ++pass) {
    if (pass > 0)
      BBX_LAUNCH("pair_hist_mid", k_lab_hist<false>, bp.g_lv[k] < 2048 ? bp.g_lv[k] : 2048, kBlock,
                 0, s, k + 1, pass, bp.nsets, plv, w.sets, w.params, K0, K1, w.labels, w.sel,
                 w.hist, w.rows, w.pass_need);
    BBX_LAUNCH("pair_select_mid", k_select_mid, sel_grid(bp.g_nd[k + 1]), kBlock, 0, s, k + 1, pass,
               1u, bp.nsets, pnd2, w.sets, w.params, w.sel, w.hist, w.pass_need);
  }
  BBX_LAUNCH("pair_hist_last", k_lab_hist<true>, bp.g_lv[k], kBlock, 0, s, k + 1, 0u, bp.nsets, plv,
             w.sets, w.params, K0, K1, w.labels, w.sel, w.hist, w.rows, w.pass_need);
  if (bp.pair_wide[k])
    BBX_LAUNCH("pair_select_last", k_select_last_wide,
               bp.g_nd[k + 1] < 8192 ? (bp.g_nd[k + 1] ? bp.g_nd[k + 1] : 1) : 8192, kBlock, 0, s,
               k + 1, 1u, bp.nsets, pnd2, w.sets, w.params, w.sel, w.hist, w.rows, w.chunk_base);
  else
    BBX_LAUNCH("pair_select_last", k_select_last, sel_grid(bp.g_nd[k + 1]), kBlock, 0, s, k + 1, 1u,
               bp.nsets, pnd2, w.sets, w.params, w.sel, w.hist, w.rows, w.chunk_base);
  BBX_LAUNCH("pair_scatter", bp.track ? k_scatter4<true> : k_scatter4<false>, bp.g_lv[k], kBlock, 0,
             s, k, bp.nsets, plv, w.sets, w.params, w.sel, w.chunk_base, K0, K1, w.idx[0], w.idx[1],
             w.hist);
  return hipGetLastError();
}

hipError_t launch_levels(const BatchPlan& bp, const Ws& w, hipStream_t s) {
  if (bp.max_gl == 0) return hipGetLastError();
  BBX_LAUNCH("level_pass_flags", k_pass_flags, 1, kBlock, 0, s, bp.nsets, w.sets, w.params,
             w.pass_need);
  // every level kernel gets buffer 0 and buffer 1 and picks, per set, the
  // one that holds the codes (paired levels shift it)
  uint8_t* K0 = w.keys[0];
  uint8_t* K1 = w.keys[1];
  uint32_t* I0 = w.idx[0];
  uint32_t* I1 = w.idx[1];
  for (uint32_t k = 0; k < bp.max_gl; ++k) {
    const uint64_t* plv = w.pre + bp.o_lv[k];
    const uint64_t* pnd = w.pre + bp.o_nd[k];
    if (bp.lv_local[k])
      BBX_LAUNCH("level_local", k_level_local, bp.g_lc[k], kBlock, 0, s, k, bp.nsets,
                 w.pre + bp.o_lc[k], w.sets, w.params, K0, K1, I0, I1, w.hist);
    if (bp.lv_wave[k])
      BBX_LAUNCH("level_wave", bp.track ? k_level_wave<true> : k_level_wave<false>,
                 (bp.g_wv[k] + kBlock / 64 - 1) / (kBlock / 64), kBlock, 0, s, k, bp.nsets,
                 w.pre + bp.o_wv[k], w.sets, w.params, K0, K1, I0, I1);
    // levels k and k + 1 in place
    if (bp.lv_fused[k])
      BBX_LAUNCH("level_fused", (bp.track ? k_level_fused<true, 1> : k_level_fused<false, 1>),
                 (bp.g_fu[k] + kBlock / 64 - 1) / (kBlock / 64), kBlock, 0, s, k, bp.nsets,
                 w.pre + bp.o_fu[k], w.sets, w.params, K0, K1, I0, I1);
    if (bp.lv_fused4[k])
      BBX_LAUNCH("level_fused4", (bp.track ? k_level_fused<true, 4> : k_level_fused<false, 4>),
                 bp.g_f4[k], kBlock, 0, s, k, bp.nsets, w.pre + bp.o_f4[k], w.sets, w.params, K0,
                 K1, I0, I1);
    if (bp.lv_fused16[k])
      BBX_LAUNCH("level_fused16", (bp.track ? k_level_fused<true, 16> : k_level_fused<false, 16>),
                 bp.g_f16[k], fused_threads<16>(), 0, s, k, bp.nsets, w.pre + bp.o_f16[k], w.sets,
                 w.params, K0, K1, I0, I1);
    if (!bp.lv_global[k]) continue;
    // mid passes: pass 0 was built by the quantize pass (depth 0) or by the
    // previous scatter
    for (uint32_t pass = 0; pass < 3; ++pass) {
      if (pass > 0)
        BBX_LAUNCH("level_hist_mid", k_hist_mid, bp.g_lv[k] < 2048 ? bp.g_lv[k] : 2048, kBlock, 0, s,
                   k, pass, bp.nsets, plv, w.sets, w.params, K0, K1, w.sel, w.hist, w.pass_need);
      BBX_LAUNCH("level_select_mid", k_select_mid, sel_grid(bp.g_nd[k]), kBlock, 0, s, k, pass, 0u,
                 bp.nsets, pnd, w.sets, w.params, w.sel, w.hist, w.pass_need);
    }
    BBX_LAUNCH("level_hist_last", k_hist_last, bp.g_lv[k], kBlock, 0, s, k, bp.nsets, plv, w.sets,
               w.params, K0, K1, w.sel, w.hist, w.rows);
    if (bp.sel_wide[k])  // some set's nodes have many chunks at this level
      BBX_LAUNCH("level_select_last", k_select_last_wide,
                 bp.g_nd[k] < 8192 ? (bp.g_nd[k] ? bp.g_nd[k] : 1) : 8192, kBlock, 0, s, k, 0u,
                 bp.nsets, pnd, w.sets, w.params, w.sel, w.hist, w.rows, w.chunk_base);
    else
      BBX_LAUNCH("level_select_last", k_select_last, sel_grid(bp.g_nd[k]), kBlock, 0, s, k, 0u,
                 bp.nsets, pnd, w.sets, w.params, w.sel, w.hist, w.rows, w.chunk_base);
    if (bp.lv_single[k])
      BBX_LAUNCH("level_scatter",
                 (bp.track ? (bp.scat_stage[k] ? k_scatter<true, true> : k_scatter<true, false>)
                           : (bp.scat_stage[k] ? k_scatter<false, true> : k_scatter<false, false>)),
                 bp.g_lv[k], kBlock, 0, s, k, bp.nsets, plv, w.sets, w.params, w.sel, w.chunk_base,
                 K0, K1, I0, I1, w.hist);
    if (bp.lv_pair[k]) {
      const hipError_t e = launch_pair(bp, w, k, s);
      if (e != hipSuccess) return e;
    }
  }
  return hipGetLastError();
}

}  // namespace bbx

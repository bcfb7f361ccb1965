// k_tile.hip -- the on-chip stage of the k-d partition plus the per-leaf bit
// box (Sec. 4.1), and the equivalent stage for leaves larger than a tile.
//
// k_tile: one workgroup per node of the tile depth (<= TILE particles).  The
// node's keys are staged in LDS once; every remaining level is a radix select
// over LDS histograms followed by a stable partition of a u16 position
// permutation (the keys themselves never move in LDS).  Then one wavefront per
// leaf computes the AABB, the reference (member nearest the AABB centre,
// squared distance in doubled code space, ties to the first member), Eq. 2's
// widths m_d = bitlen(D_d) + 1 (0 when D_d = 0), and writes the leaf's keys
// back in output-slot order (reference first) together with its record.
//
// k_bigleaf: one workgroup per leaf when leaves exceed the tile capacity.
#include "bbx_internal.h"

namespace bbx {

__device__ inline uint32_t wmin_u32(uint32_t v) {
  for (int o = 32; o > 0; o >>= 1) {
    uint32_t u = __shfl_xor(v, o);
    v = u < v ? u : v;
  }
  return v;
}
__device__ inline uint32_t wmax_u32(uint32_t v) {
  for (int o = 32; o > 0; o >>= 1) {
    uint32_t u = __shfl_xor(v, o);
    v = u > v ? u : v;
  }
  return v;
}
// (dist, pos) minimum: smaller distance, then smaller position
__device__ inline void wargmin(uint64_t& dist, uint32_t& pos) {
  for (int o = 32; o > 0; o >>= 1) {
    uint64_t d2 = __shfl_xor(dist, o);
    uint32_t p2 = __shfl_xor(pos, o);
    if (d2 < dist || (d2 == dist && p2 < pos)) dist = d2, pos = p2;
  }
}

__device__ inline uint32_t width_of(uint32_t D) { return D ? bitlen32(D) + 1u : 0u; }

__device__ inline uint64_t sqdist3(const uint32_t* q, const uint32_t* C, uint32_t dims) {
  uint64_t s = 0;
  for (uint32_t d = 0; d < dims; ++d) {
    int64_t t = 2 * (int64_t)q[d] - (int64_t)C[d];
    s += (uint64_t)(t * t);
  }
  return s;
}

template <int TILE>
struct TileSmem {
  uint32_t K[3][TILE];
  uint16_t Pm[2][TILE];
  uint32_t I[TILE];
  uint32_t H[2048];
  uint32_t S[TILE];
  uint16_t nst[TILE / 2], nsz[TILE / 2];
  uint32_t npre[TILE / 2], nrank[TILE / 2];
  uint32_t wsum[kBlock / 64];
  uint32_t nleaves;
};

template <int TILE>
__device__ inline uint32_t find_node(const TileSmem<TILE>& sm, uint32_t N, uint32_t p) {
  uint32_t lo = 0, hi = N - 1;  // largest i with nst[i] <= p
  while (lo < hi) {
    uint32_t mid = (lo + hi + 1) >> 1;
    if (sm.nst[mid] <= p)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// block exclusive scan of u32 (256 threads)
template <int TILE>
__device__ inline uint32_t tile_exscan(TileSmem<TILE>& sm, uint32_t v) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t x = v;
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) sm.wsum[wv] = x;
  __syncthreads();
  uint32_t off = 0;
  for (int k = 0; k < wv; ++k) off += sm.wsum[k];
  __syncthreads();
  return off + x - v;
}

template <int TILE, typename KT>
__device__ void tile_body(TileSmem<TILE>& sm, uint32_t K0, uint64_t n, uint32_t dims, uint32_t r,
                          uint64_t n_leaves, const TreeGeom& g, DevParams* P, KT* keys,
                          const uint32_t* idx,
                          uint32_t* perm, LeafRec* leaves, uint64_t* leaf_bits) {
  constexpr int ITEMS = TILE / kBlock;
  const uint64_t j = blockIdx.x;
  uint64_t tst, s0_64;
  node_span(n, K0, j, &tst, &s0_64);
  if (s0_64 > (uint64_t)TILE) {  // launch plan violated: never expected
    if (threadIdx.x == 0) P->status = BBX_EHIP;
    return;
  }
  const uint32_t s0 = (uint32_t)s0_64;
  const uint64_t first_leaf = leaves_before_node(g, K0, j, tst);
  const bool track = idx != nullptr;

  for (uint32_t d = 0; d < dims; ++d)
    for (uint32_t p = threadIdx.x; p < s0; p += kBlock) sm.K[d][p] = keys[(uint64_t)d * n + tst + p];
  for (uint32_t p = threadIdx.x; p < s0; p += kBlock) {
    sm.Pm[0][p] = (uint16_t)p;
    if (track) sm.I[p] = idx[tst + p];
  }
  __syncthreads();

  int cur = 0;
  int last_l = -1;
  uint32_t lastN = 0;
  for (uint32_t l = 0;; ++l) {
    const uint32_t N = 1u << l;
    const uint32_t maxsz = (s0 + N - 1) >> l;
    if (maxsz <= r) break;
    const uint32_t d = (K0 + l) % dims;
    const uint32_t G = P->G[d];
    for (uint32_t i = threadIdx.x; i < N; i += kBlock) {
      uint64_t a, b;
      node_span(s0, l, i, &a, &b);
      sm.nst[i] = (uint16_t)a;
      sm.nsz[i] = (uint16_t)b;
      sm.npre[i] = 0;
      sm.nrank[i] = (uint32_t)(b >> 1);
    }
    __syncthreads();
    // ---- radix select of each internal node's median code
    const uint32_t Wl = (11u - l) < 8u ? (11u - l) : 8u;
    const uint32_t npass = G == 0 ? 1u : (G + Wl - 1) / Wl;
    const uint32_t firstw = G - (npass - 1) * Wl;
    const uint32_t p0 = threadIdx.x * ITEMS;
    uint32_t used = 0;
    for (uint32_t pass = 0; pass < npass; ++pass) {
      const uint32_t w = pass == 0 ? firstw : Wl;
      const uint32_t hs = G - used;
      used += w;
      const uint32_t sh = G - used;
      const uint32_t nb = 1u << w, mask = nb - 1;
      for (uint32_t b = threadIdx.x; b < (N << w); b += kBlock) sm.H[b] = 0;
      __syncthreads();
      if (p0 < s0) {
        uint32_t i = find_node(sm, N, p0);
        for (int k = 0; k < ITEMS; ++k) {
          uint32_t p = p0 + k;
          if (p >= s0) break;
          while (p >= (uint32_t)sm.nst[i] + sm.nsz[i]) ++i;
          if (sm.nsz[i] <= r) continue;
          uint32_t q = sm.K[d][sm.Pm[cur][p]];
          if ((hs >= 32 ? 0u : (q >> hs)) == sm.npre[i]) atomicAdd(&sm.H[(i << w) + ((q >> sh) & mask)], 1u);
        }
      }
      __syncthreads();
      // wave per node: find the bin holding the rank
      const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
      for (uint32_t i = wv; i < N; i += kBlock / 64) {
        if (sm.nsz[i] <= r) continue;
        const uint32_t per = (nb + 63) / 64;  // <= 4
        uint32_t c[4] = {0, 0, 0, 0};
        uint32_t mine = 0;
        for (uint32_t k = 0; k < per; ++k) {
          uint32_t b = lane * per + k;
          c[k] = b < nb ? sm.H[(i << w) + b] : 0u;
          mine += c[k];
        }
        uint32_t x = mine;
        for (int o = 1; o < 64; o <<= 1) {
          uint32_t y = __shfl_up(x, o);
          if (lane >= o) x += y;
        }
        uint32_t cum = x - mine;
        const uint32_t rank = sm.nrank[i];
        const uint32_t pre = sm.npre[i];
        for (uint32_t k = 0; k < per; ++k) {
          if (cum <= rank && rank < cum + c[k]) {
            sm.npre[i] = (pre << w) | (lane * per + k);
            sm.nrank[i] = rank - cum;
          }
          cum += c[k];
        }
      }
      __syncthreads();
    }
    // ---- stable partition: exclusive prefix of (lt | eq << 16) over the tile
    uint32_t fl[ITEMS];
    uint32_t mine = 0;
    {
      uint32_t i = p0 < s0 ? find_node(sm, N, p0) : 0;
      for (int k = 0; k < ITEMS; ++k) {
        uint32_t p = p0 + k;
        fl[k] = 0;
        if (p >= s0) continue;
        while (p >= (uint32_t)sm.nst[i] + sm.nsz[i]) ++i;
        if (sm.nsz[i] > r) {
          uint32_t q = sm.K[d][sm.Pm[cur][p]];
          uint32_t v = sm.npre[i];
          fl[k] = (q < v ? 1u : 0u) | (q == v ? 0x10000u : 0u);
        }
        mine += fl[k];
      }
    }
    uint32_t ex = tile_exscan(sm, mine);
    for (int k = 0; k < ITEMS; ++k) {
      uint32_t p = p0 + k;
      if (p < s0) sm.S[p] = ex;
      ex += fl[k];
    }
    __syncthreads();
    if (p0 < s0) {
      uint32_t i = find_node(sm, N, p0);
      for (int k = 0; k < ITEMS; ++k) {
        uint32_t p = p0 + k;
        if (p >= s0) break;
        while (p >= (uint32_t)sm.nst[i] + sm.nsz[i]) ++i;
        const uint32_t ns = sm.nst[i], nz = sm.nsz[i];
        if (nz <= r) {
          sm.Pm[cur ^ 1][p] = sm.Pm[cur][p];
          continue;
        }
        const uint32_t X = sm.S[p] - sm.S[ns];
        const uint32_t L = X & 0xffffu, E = X >> 16;
        const uint32_t jeq = sm.nrank[i];
        const uint32_t lb = L + (E < jeq ? E : jeq);
        const bool lt = fl[k] & 1u, eq = (fl[k] >> 16) & 1u;
        const bool left = lt || (eq && E < jeq);
        const uint32_t dest = left ? lb : (nz >> 1) + (p - ns) - lb;
        if (dest < nz) sm.Pm[cur ^ 1][ns + dest] = sm.Pm[cur][p];
      }
    }
    __syncthreads();
    cur ^= 1;
    last_l = (int)l;
    lastN = N;
  }

  // ---- leaf list (depth-first): nodes of the last level that were split give
  // two leaves, the others are leaves themselves
  if (last_l < 0) {
    if (threadIdx.x == 0) {
      sm.H[0] = 0u | ((uint32_t)s0 << 16);
      sm.nleaves = 1;
    }
  } else {
    const uint32_t N = lastN;
    const uint32_t per = (N + kBlock - 1) / kBlock;  // <= 4
    uint32_t cnt = 0;
    for (uint32_t k = 0; k < per; ++k) {
      uint32_t i = threadIdx.x * per + k;
      if (i < N) cnt += sm.nsz[i] > r ? 2u : 1u;
    }
    uint32_t at = tile_exscan(sm, cnt);
    for (uint32_t k = 0; k < per; ++k) {
      uint32_t i = threadIdx.x * per + k;
      if (i >= N) break;
      const uint32_t ns = sm.nst[i], nz = sm.nsz[i];
      if (nz > r) {
        sm.H[at++] = ns | ((nz >> 1) << 16);
        sm.H[at++] = (ns + (nz >> 1)) | ((nz - (nz >> 1)) << 16);
      } else {
        sm.H[at++] = ns | (nz << 16);
      }
    }
    if (threadIdx.x == kBlock - 1) sm.nleaves = at;
  }
  __syncthreads();

  // ---- bit box per leaf, one wavefront each
  const uint32_t nl = sm.nleaves;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (uint32_t L = wv; L < nl; L += kBlock / 64) {
    const uint32_t ls = sm.H[L] & 0xffffu, lz = sm.H[L] >> 16;
    uint32_t mn[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu}, mx[3] = {0, 0, 0};
    for (uint32_t t = lane; t < lz; t += 64) {
      const uint32_t slot = sm.Pm[cur][ls + t];
      for (uint32_t d = 0; d < dims; ++d) {
        uint32_t q = sm.K[d][slot];
        mn[d] = q < mn[d] ? q : mn[d];
        mx[d] = q > mx[d] ? q : mx[d];
      }
    }
    uint32_t C[3] = {0, 0, 0};
    for (uint32_t d = 0; d < dims; ++d) {
      mn[d] = wmin_u32(mn[d]);
      mx[d] = wmax_u32(mx[d]);
      C[d] = mn[d] + mx[d];
    }
    uint64_t best = ~0ull;
    uint32_t bpos = 0xffffffffu;
    for (uint32_t t = lane; t < lz; t += 64) {
      const uint32_t slot = sm.Pm[cur][ls + t];
      uint32_t q[3] = {0, 0, 0};
      for (uint32_t d = 0; d < dims; ++d) q[d] = sm.K[d][slot];
      uint64_t dist = sqdist3(q, C, dims);
      if (dist < best) best = dist, bpos = t;  // t increases: ties keep the first
    }
    wargmin(best, bpos);
    const uint32_t ref = bpos;
    const uint32_t rslot = sm.Pm[cur][ls + ref];
    uint32_t m[3] = {0, 0, 0}, qr[3] = {0, 0, 0};
    uint32_t summ = 0;
    for (uint32_t d = 0; d < dims; ++d) {
      qr[d] = sm.K[d][rslot];
      uint32_t D = (qr[d] - mn[d]) > (mx[d] - qr[d]) ? qr[d] - mn[d] : mx[d] - qr[d];
      m[d] = width_of(D);
      summ += m[d];
    }
    const uint64_t lid = first_leaf + L;
    if (lid >= n_leaves) continue;  // leaf count mismatch: never expected
    if (lane == 0) {
      LeafRec rec;
      rec.start = (uint32_t)(tst + ls);
      rec.size = lz;
      rec.m = m[0] | (m[1] << 8) | (m[2] << 16);
      rec.qref[0] = qr[0];
      rec.qref[1] = qr[1];
      rec.qref[2] = qr[2];
      leaves[lid] = rec;
      leaf_bits[lid] = (uint64_t)(lz - 1) * summ;
    }
    for (uint32_t t = lane; t < lz; t += 64) {
      const uint32_t slot = sm.Pm[cur][ls + t];
      const uint32_t o = t == ref ? 0u : (t < ref ? t + 1 : t);
      const uint64_t gpos = tst + ls + o;
      for (uint32_t d = 0; d < dims; ++d) keys[(uint64_t)d * n + gpos] = (KT)sm.K[d][slot];
      if (track) perm[gpos] = sm.I[slot];
    }
  }
}

template <int TILE>
__global__ void __launch_bounds__(kBlock) k_tile(uint32_t K0, uint64_t n, uint32_t dims,
                                                 uint32_t r, uint64_t n_leaves, TreeGeom g,
                                                 DevParams* P,
                                                 void* keys, const uint32_t* idx, uint32_t* perm,
                                                 LeafRec* leaves, uint64_t* leaf_bits) {
  if (P->status != BBX_OK) return;
  __shared__ TileSmem<TILE> sm;
  if (P->key16)
    tile_body<TILE, uint16_t>(sm, K0, n, dims, r, n_leaves, g, P, (uint16_t*)keys, idx, perm, leaves,
                              leaf_bits);
  else
    tile_body<TILE, uint32_t>(sm, K0, n, dims, r, n_leaves, g, P, (uint32_t*)keys, idx, perm, leaves,
                              leaf_bits);
}

// ---------------------------------------------------------------- big leaves

__device__ inline uint32_t bmin_u32(uint32_t v, uint32_t* red) {
  v = wmin_u32(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) red[wv] = v;
  __syncthreads();
  uint32_t r = red[0];
  for (int k = 1; k < kBlock / 64; ++k) r = red[k] < r ? red[k] : r;
  __syncthreads();
  return r;
}
__device__ inline uint32_t bmax_u32(uint32_t v, uint32_t* red) {
  v = wmax_u32(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) red[wv] = v;
  __syncthreads();
  uint32_t r = red[0];
  for (int k = 1; k < kBlock / 64; ++k) r = red[k] > r ? red[k] : r;
  __syncthreads();
  return r;
}

template <typename KT>
__device__ void bigleaf_body(uint64_t n, uint32_t dims, const TreeGeom& g, const KT* src, KT* dst,
                             const uint32_t* idx, uint32_t* perm, LeafRec* leaves,
                             uint64_t* leaf_bits) {
  __shared__ uint32_t red[kBlock / 64];
  __shared__ uint64_t rd[kBlock / 64];
  __shared__ uint32_t rp[kBlock / 64];
  const uint64_t i = blockIdx.x;
  uint64_t st, sz;
  leaf_span(g, i, &st, &sz);
  uint32_t mn[3] = {0, 0, 0}, mx[3] = {0, 0, 0}, C[3] = {0, 0, 0};
  for (uint32_t d = 0; d < dims; ++d) {
    uint32_t a = 0xffffffffu, b = 0;
    for (uint64_t p = threadIdx.x; p < sz; p += kBlock) {
      uint32_t q = src[(uint64_t)d * n + st + p];
      a = q < a ? q : a;
      b = q > b ? q : b;
    }
    mn[d] = bmin_u32(a, red);
    mx[d] = bmax_u32(b, red);
    C[d] = mn[d] + mx[d];
  }
  uint64_t best = ~0ull;
  uint32_t bpos = 0xffffffffu;
  for (uint64_t p = threadIdx.x; p < sz; p += kBlock) {
    uint32_t q[3] = {0, 0, 0};
    for (uint32_t d = 0; d < dims; ++d) q[d] = src[(uint64_t)d * n + st + p];
    uint64_t dist = sqdist3(q, C, dims);
    if (dist < best) best = dist, bpos = (uint32_t)p;
  }
  wargmin(best, bpos);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) rd[wv] = best, rp[wv] = bpos;
  __syncthreads();
  best = rd[0];
  bpos = rp[0];
  for (int k = 1; k < kBlock / 64; ++k)
    if (rd[k] < best || (rd[k] == best && rp[k] < bpos)) best = rd[k], bpos = rp[k];
  const uint32_t ref = bpos;
  uint32_t m[3] = {0, 0, 0}, qr[3] = {0, 0, 0}, summ = 0;
  for (uint32_t d = 0; d < dims; ++d) {
    qr[d] = src[(uint64_t)d * n + st + ref];
    uint32_t D = (qr[d] - mn[d]) > (mx[d] - qr[d]) ? qr[d] - mn[d] : mx[d] - qr[d];
    m[d] = width_of(D);
    summ += m[d];
  }
  if (threadIdx.x == 0) {
    LeafRec rec;
    rec.start = (uint32_t)st;
    rec.size = (uint32_t)sz;
    rec.m = m[0] | (m[1] << 8) | (m[2] << 16);
    rec.qref[0] = qr[0];
    rec.qref[1] = qr[1];
    rec.qref[2] = qr[2];
    leaves[i] = rec;
    leaf_bits[i] = (sz - 1) * (uint64_t)summ;
  }
  for (uint64_t p = threadIdx.x; p < sz; p += kBlock) {
    const uint64_t o = p == ref ? 0 : (p < ref ? p + 1 : p);
    for (uint32_t d = 0; d < dims; ++d) dst[(uint64_t)d * n + st + o] = src[(uint64_t)d * n + st + p];
    if (idx) perm[st + o] = idx[st + p];
  }
}

__global__ void __launch_bounds__(kBlock) k_bigleaf(uint64_t n, uint32_t dims, TreeGeom g,
                                                    const DevParams* P, const void* src,
                                                    void* dst, const uint32_t* idx,
                                                    uint32_t* perm, LeafRec* leaves,
                                                    uint64_t* leaf_bits) {
  if (P->status != BBX_OK) return;
  if (P->key16)
    bigleaf_body<uint16_t>(n, dims, g, (const uint16_t*)src, (uint16_t*)dst, idx, perm, leaves,
                           leaf_bits);
  else
    bigleaf_body<uint32_t>(n, dims, g, (const uint32_t*)src, (uint32_t*)dst, idx, perm, leaves,
                           leaf_bits);
}

hipError_t launch_leaves(const CompressPlan& p, const CompressWs& w, int buf, uint32_t* perm,
                         hipStream_t s, int* out_buf) {
  const uint32_t* idx = p.track_idx ? w.idx[buf] : nullptr;
  if (p.tile_mode) {
    const uint64_t tiles = 1ull << p.global_levels;
    if (p.tile == 1024)
      BBX_LAUNCH("tile", k_tile<1024>, tiles, kBlock, 0, s, p.global_levels, p.n, p.dims, p.r,
                 p.n_leaves, p.geom, w.params, w.keys[buf], idx, perm, w.leaves, w.leaf_bits);
    else
      BBX_LAUNCH("tile", k_tile<2048>, tiles, kBlock, 0, s, p.global_levels, p.n, p.dims, p.r,
                 p.n_leaves, p.geom, w.params, w.keys[buf], idx, perm, w.leaves, w.leaf_bits);
    *out_buf = buf;
  } else {
    BBX_LAUNCH("bigleaf", k_bigleaf, p.n_leaves, kBlock, 0, s, p.n, p.dims, p.geom, w.params,
               w.keys[buf], w.keys[buf ^ 1], idx, perm, w.leaves, w.leaf_bits);
    *out_buf = buf ^ 1;
  }
  return hipGetLastError();
}

}  // namespace bbx

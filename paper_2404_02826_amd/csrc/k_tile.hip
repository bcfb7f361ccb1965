// k_tile.hip -- the on-chip stage of the k-d partition plus the per-leaf bit
// box (Sec. 4.1), and the equivalent stage for leaves larger than a tile.
//
// k_tile: one wavefront per node of the tile depth (<= TILE particles), with
// no workgroup barriers: the node's codes are staged in the wavefront's own
// LDS slice once, and LDS operations of one wavefront complete in program
// order.  Every remaining level is a radix select over LDS histograms
// followed by a stable partition of a u16 position permutation (the codes
// never move in LDS).  Leaves are then handled by aligned lane groups (a
// power of two >= the leaf size, up to the wavefront): AABB, reference =
// member nearest the AABB centre (squared distance in doubled code space) or,
// with reference rule 1, the member with the smallest sum of Eq. 2 widths
// (ties to the first member either way), Eq. 2's widths m_d = bitlen(D_d) + 1
// (0 when D_d = 0).  Finally the node is written back in output-slot order (reference
// first in each leaf) with coalesced stores.
//
// k_bigleaf: one workgroup per leaf when leaves exceed the tile capacity.
#include <type_traits>

#include "bbx_internal.h"

namespace bbx {

// reductions within aligned groups of gs lanes (gs a power of two <= 64)
__device__ inline uint32_t gmin_u32(uint32_t v, uint32_t gs) {
  for (uint32_t o = gs >> 1; o > 0; o >>= 1) {
    uint32_t u = __shfl_xor(v, (int)o);
    v = u < v ? u : v;
  }
  return v;
}
__device__ inline uint32_t gmax_u32(uint32_t v, uint32_t gs) {
  for (uint32_t o = gs >> 1; o > 0; o >>= 1) {
    uint32_t u = __shfl_xor(v, (int)o);
    v = u > v ? u : v;
  }
  return v;
}
// (dist, pos) minimum: smaller distance, then smaller position
__device__ inline void gargmin(uint64_t& dist, uint32_t& pos, uint32_t gs) {
  for (uint32_t o = gs >> 1; o > 0; o >>= 1) {
    uint64_t d2 = __shfl_xor(dist, (int)o);
    uint32_t p2 = __shfl_xor(pos, (int)o);
    if (d2 < dist || (d2 == dist && p2 < pos)) dist = d2, pos = p2;
  }
}
// the same over aligned groups of 8 lanes by DPP moves: neighbours, then
// pairs within the quad, then the group's other quad through the half-row
// mirror (lane i of a half-row reads lane 7 - i)
template <typename F>
__device__ __forceinline__ uint32_t g8_reduce(uint32_t v, F&& op) {
  v = op(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0xB1, 0xf, 0xf, false));   // quad_perm 1,0,3,2
  v = op(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x4E, 0xf, 0xf, false));   // quad_perm 2,3,0,1
  v = op(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x141, 0xf, 0xf, false));  // row_half_mirror
  return v;
}
__device__ inline uint32_t wmin_u32(uint32_t v) { return gmin_u32(v, 64); }
__device__ inline uint32_t wmax_u32(uint32_t v) { return gmax_u32(v, 64); }
__device__ inline void wargmin(uint64_t& dist, uint32_t& pos) { gargmin(dist, pos, 64); }

__device__ inline uint32_t width_of(uint32_t D) { return D ? bitlen32(D) + 1u : 0u; }

__device__ inline uint64_t sqdist3(const uint32_t* q, const uint32_t* C, uint32_t dims) {
  uint64_t s = 0;
  for (uint32_t d = 0; d < dims; ++d) {
    int64_t t = 2 * (int64_t)q[d] - (int64_t)C[d];
    s += (uint64_t)(t * t);
  }
  return s;
}

// LDS of one tile.  KL holds codes minus the tile's per-axis minimum: 16 bits
// for every tile whose spans fit (the first pass), 32 bits for the rest (a
// second pass over the tiles the first one deferred).  Source indices only
// take space when some set asks for a perm output.
template <int TILE, typename KL, bool TRACK>
struct WaveTile {
  KL K[3][TILE];                 // codes minus the tile minimum, at original slots
  uint16_t Pm[2][TILE];          // position -> slot (ping-pong)
  uint32_t I[TRACK ? TILE : 1];  // source indices
  uint32_t H[TILE];              // histogram bins (all zero between passes); then the leaf table
  uint32_t S[TILE];              // exclusive (lt | eq << 16) prefix; then position -> leaf
  uint16_t nst[TILE / 2], nsz[TILE / 2];
  KL npre[TILE / 2];             // high digits of each node's median found so far
  uint16_t nrank[TILE / 2];      // rank of the median among the remaining candidates
  uint16_t lref[TILE];           // reference position within each leaf
};

__device__ inline uint32_t leaf_fold(uint32_t s, uint32_t r) { return s <= r ? s : s - (s >> 1); }

// Bit boxes of the tile's leaves (Sec. 4.1, Eq. 2) by aligned groups of gs
// lanes; DT holds squared distances in doubled code space (32 bits suffice
// when every code span is below 2^14).  With M > 0 every leaf has at most
// M * gs members: each lane reads its members' codes once into registers
// (fixed trip counts); M = 0 walks the members from LDS in each pass.
template <int TILE, typename KL, bool TRACK, typename DT, int M, int GS = 0>
__device__ void tile_bitboxes(WaveTile<TILE, KL, TRACK>& sm, int cur, uint32_t nl, uint32_t gs_rt, uint32_t dims,
                              uint32_t t0, uint32_t t1, uint32_t t2, uint64_t tst, uint64_t first_leaf,
                              uint64_t n_leaves, DevParams* P, LeafRec* leaves,
                              uint64_t* leaf_bits, uint32_t rule) {
  constexpr int MR = M > 0 ? M : 1;
  static_assert(GS == 0 || GS == 8, "groups of 8 lanes or of a run-time size");
  const uint32_t gs = GS ? (uint32_t)GS : gs_rt;  // GS: the group size, fixed at compile time
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t lpw = 64 / gs;
  const uint32_t sub = lane & (gs - 1);
  for (uint32_t base = 0; base < nl; base += lpw) {
    const uint32_t L = base + lane / gs;
    const bool act = L < nl;
    const uint32_t ls = act ? (sm.H[L] & 0xffffu) : 0u, lz = act ? (sm.H[L] >> 16) : 0u;
    uint32_t mn[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu}, mx[3] = {0, 0, 0};
    uint32_t rq[3][MR];  // M > 0: the lane's members (member sub + gs * m)
    if (M > 0) {
#pragma unroll
      for (int m = 0; m < MR; ++m) {
        const uint32_t t = sub + gs * (uint32_t)m;
        const uint32_t slot = t < lz ? sm.Pm[cur][ls + t] : 0u;
#pragma unroll
        for (uint32_t d = 0; d < 3; ++d) {
          rq[d][m] = d < dims ? (uint32_t)sm.K[d][slot] : 0u;
          if (t < lz) {
            mn[d] = umin32(rq[d][m], mn[d]);
            mx[d] = umax32(rq[d][m], mx[d]);
          }
        }
      }
    } else {
      for (uint32_t t = sub; t < lz; t += gs) {
        const uint32_t slot = sm.Pm[cur][ls + t];
#pragma unroll
        for (uint32_t d = 0; d < 3; ++d) {
          if (d >= dims) break;
          const uint32_t q = sm.K[d][slot];
          mn[d] = umin32(q, mn[d]);
          mx[d] = umax32(q, mx[d]);
        }
      }
    }
    DT C[3] = {0, 0, 0};
#pragma unroll
    for (uint32_t d = 0; d < 3; ++d) {
      if (d >= dims) break;
      if constexpr (GS == 8) {
        mn[d] = g8_reduce(mn[d], [](uint32_t a, uint32_t b) { return umin32(a, b); });
        mx[d] = g8_reduce(mx[d], [](uint32_t a, uint32_t b) { return umax32(a, b); });
      } else {
        mn[d] = gmin_u32(mn[d], gs);
        mx[d] = gmax_u32(mx[d], gs);
      }
      C[d] = (DT)mn[d] + (DT)mx[d];
    }
    DT best = (DT)~(DT)0;
    uint32_t bpos = 0xffffffffu;
    // candidate distance of a member with codes q (Eq. 2 widths with rule 1)
    auto dist_of = [&](const uint32_t* q) -> DT {
      DT dist = 0;
      if (rule) {  // fewest code bits: sum_d m_d with this member as the reference
        uint32_t bits = 0;
#pragma unroll
        for (uint32_t d = 0; d < 3; ++d) {
          if (d >= dims) break;
          bits += width_of(umax32(q[d] - mn[d], mx[d] - q[d]));
        }
        dist = (DT)bits;
      } else {  // nearest the AABB centre
#pragma unroll
        for (uint32_t d = 0; d < 3; ++d) {
          if (d >= dims) break;
          const DT q2 = 2 * (DT)q[d];
          const DT a = q2 > C[d] ? q2 - C[d] : C[d] - q2;
          dist += a * a;
        }
      }
      return dist;
    };
    if (M > 0) {
#pragma unroll
      for (int m = 0; m < MR; ++m) {
        const uint32_t t = sub + gs * (uint32_t)m;
        const uint32_t q[3] = {rq[0][m], rq[1][m], rq[2][m]};
        const DT dist = dist_of(q);
        if (t < lz && dist < best) best = dist, bpos = t;  // t increases: ties keep the first
      }
    } else {
      for (uint32_t t = sub; t < lz; t += gs) {
        const uint32_t slot = sm.Pm[cur][ls + t];
        uint32_t q[3] = {0, 0, 0};
#pragma unroll
        for (uint32_t d = 0; d < 3; ++d)
          if (d < dims) q[d] = sm.K[d][slot];
        const DT dist = dist_of(q);
        if (dist < best) best = dist, bpos = t;  // t increases: ties keep the first
      }
    }
    if constexpr (GS == 8 && sizeof(DT) == 4) {
      auto take = [&](auto ctrl_tag) __attribute__((always_inline)) {
        constexpr int ctrl = decltype(ctrl_tag)::value;
        const DT d2 = (DT)__builtin_amdgcn_update_dpp((int)best, (int)best, ctrl, 0xf, 0xf, false);
        const uint32_t p2 = (uint32_t)__builtin_amdgcn_update_dpp((int)bpos, (int)bpos, ctrl, 0xf, 0xf, false);
        if (d2 < best || (d2 == best && p2 < bpos)) best = d2, bpos = p2;
      };
      take(std::integral_constant<int, 0xB1>{});   // quad_perm 1,0,3,2
      take(std::integral_constant<int, 0x4E>{});   // quad_perm 2,3,0,1
      take(std::integral_constant<int, 0x141>{});  // row_half_mirror
    } else {
      for (uint32_t o = gs >> 1; o > 0; o >>= 1) {
        const DT d2 = __shfl_xor(best, (int)o);
        const uint32_t p2 = __shfl_xor(bpos, (int)o);
        if (d2 < best || (d2 == best && p2 < bpos)) best = d2, bpos = p2;
      }
    }
    if (!act) continue;
    const uint32_t ref = bpos;
    if constexpr (GS > 0 && M > 0) {
#pragma unroll
      for (int m = 0; m < M; ++m) {  // position -> leaf
        const uint32_t t = sub + GS * (uint32_t)m;
        if (t < lz) sm.S[ls + t] = L;
      }
    } else {
      for (uint32_t t = sub; t < lz; t += gs) sm.S[ls + t] = L;  // position -> leaf
    }
    if (sub == 0) {
      const uint32_t rslot = sm.Pm[cur][ls + ref];
      const uint32_t tmin[3] = {t0, t1, t2};
      uint32_t m[3] = {0, 0, 0}, qr[3] = {0, 0, 0};
      uint32_t summ = 0;
#pragma unroll
      for (uint32_t d = 0; d < 3; ++d) {
        if (d >= dims) break;
        const uint32_t q = sm.K[d][rslot];
        const uint32_t D = umax32(q - mn[d], mx[d] - q);
        m[d] = width_of(D);
        qr[d] = q + tmin[d];
        summ += m[d];
      }
      sm.lref[L] = (uint16_t)ref;
      const uint64_t lid = first_leaf + L;
      if (lid < n_leaves) {
        LeafRec rec;
        rec.start = (uint32_t)(tst + ls);
        rec.size = lz;
        rec.m = m[0] | (m[1] << 8) | (m[2] << 16);
        rec.qref[0] = qr[0];
        rec.qref[1] = qr[1];
        rec.qref[2] = qr[2];
        rec.ref_src = TRACK ? sm.I[rslot] : 0u;  // meaningful when the set carries indices
        leaves[lid] = rec;
        leaf_bits[lid] = (uint64_t)(lz - 1) * summ;
      } else {
        check_failed(P, kChkTileLeaves);  // leaf count mismatch: never expected
      }
    }
  }
}

// One node of the tile depth.  With 16-bit tile codes, a node whose code
// span along some axis exceeds 16 bits is appended to `defer` ([0] = count,
// then global tile indices) and left to the 32-bit pass.
template <int TILE, typename KT, typename KL, bool TRACK>
__device__ void tile_body(WaveTile<TILE, KL, TRACK>& sm, uint64_t j, uint32_t K0, uint64_t n,
                          uint64_t kst, uint32_t dims, uint32_t r, uint64_t n_leaves,
                          const TreeGeom& g, DevParams* P, KT* keys, const uint32_t* idx,
                          uint32_t* perm, LeafRec* leaves, uint64_t* leaf_bits, uint32_t* defer,
                          uint32_t gtile, uint32_t rule) {
  constexpr int E = TILE / 64;
  const uint32_t lane = threadIdx.x & 63;
  uint64_t tst, s0_64;
  node_span(n, K0, j, &tst, &s0_64);
  if (s0_64 > (uint64_t)TILE) {  // launch plan violated: never expected
    if (lane == 0) check_failed(P, kChkTileRange);
    return;
  }
  const uint32_t s0 = (uint32_t)s0_64;
  const uint64_t first_leaf = leaves_before_node(g, K0, j, tst);
  const bool track = idx != nullptr;

  // ---- stage the node (loads of up to 8 rows in flight) and find the tile's
  // per-axis code range: every later step works on codes minus the minimum,
  // which keeps the radix digits few and the bins spread
  static_assert(E <= 8, "all rows of the node are held in registers while staging");
  uint32_t lo[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu}, hi[3] = {0, 0, 0};
  uint32_t v[3][E];
  uint32_t ix[E];
#pragma unroll
  for (int k = 0; k < E; ++k) {
    const uint32_t p = lane + 64u * k;
#pragma unroll
    for (uint32_t d = 0; d < 3; ++d)
      v[d][k] = (p < s0 && d < dims) ? (uint32_t)keys[(uint64_t)d * kst + tst + p] : 0u;
    ix[k] = (TRACK && p < s0 && track) ? idx[tst + p] : 0u;
  }
#pragma unroll
  for (int k = 0; k < E; ++k) {
    const uint32_t p = lane + 64u * k;
    if (p < s0)
#pragma unroll
      for (uint32_t d = 0; d < 3; ++d) {
        lo[d] = umin32(lo[d], v[d][k]);
        hi[d] = umax32(hi[d], v[d][k]);
      }
  }
  uint32_t tmin[3] = {0, 0, 0}, Gt[3] = {0, 0, 0};
#pragma unroll
  for (uint32_t d = 0; d < 3; ++d) {
    if (d >= dims) break;
    tmin[d] = wave_min_dpp(lo[d]);
    Gt[d] = bitlen32(wave_max_dpp(hi[d]) - tmin[d]);
  }
  if (sizeof(KL) == 2 && umax32(Gt[0], umax32(Gt[1], Gt[2])) > 16) {
    if (lane == 0) defer[1 + atomicAdd(&defer[0], 1u)] = gtile;  // the 32-bit pass takes it
    return;
  }
#pragma unroll
  for (int k = 0; k < E; ++k) {
    const uint32_t p = lane + 64u * k;
    if (p < s0) {
#pragma unroll
      for (uint32_t d = 0; d < 3; ++d)
        if (d < dims) sm.K[d][p] = (KL)(v[d][k] - tmin[d]);
      sm.Pm[0][p] = (uint16_t)p;
      if (TRACK && track) sm.I[p] = ix[k];
    }
    sm.H[p] = 0;
  }
  wave_sync();

  int cur = 0;
  int last_l = -1;
  uint32_t lastN = 0;
  const uint32_t p0 = lane * E;
  // The levels.  POW2: a tile of exactly TILE members and r a power of two,
  // so every node of level l holds TILE >> l members starting at a multiple
  // of that: a position's node and its bounds are shifts, every node above
  // the leaves splits, and a node's prefix at its start (a lane boundary
  // while nodes hold >= E members) comes from the first lane of the node.
  auto levels = [&](auto pow2_tag) __attribute__((always_inline)) {
    constexpr bool POW2 = decltype(pow2_tag)::value;
    constexpr uint32_t LT = TILE == 256 ? 8u : 9u;  // log2(TILE)
    // the lane's E consecutive positions: node start and size at the current
    // level, followed from level to level (a node's left child keeps the first
    // floor(s/2) positions)
    uint32_t nsr[E], nzz[E], ni[E];
#pragma unroll
    for (int k = 0; k < E; ++k) nsr[k] = 0, nzz[k] = s0, ni[k] = 0;
    for (uint32_t l = 0;; ++l) {
      const uint32_t N = 1u << l;
      const uint32_t maxsz = POW2 ? (TILE >> l) : (s0 + N - 1) >> l;
      if (maxsz <= r) break;
      const uint32_t d = (K0 + l) % dims;
      const uint32_t G = d == 0 ? Gt[0] : (d == 1 ? Gt[1] : Gt[2]);
      for (uint32_t i = lane; i < N; i += 64) {
        uint64_t a, b;
        if (POW2) {
          a = (uint64_t)i << (LT - l);
          b = TILE >> l;
        } else {
          node_span(s0, l, i, &a, &b);
        }
        sm.nst[i] = (uint16_t)a;
        sm.nsz[i] = (uint16_t)b;
        sm.npre[i] = 0;
        sm.nrank[i] = (uint16_t)(b >> 1);
      }
      if (POW2) {
#pragma unroll
        for (int k = 0; k < E; ++k) {
          ni[k] = (p0 + k) >> (LT - l);
          nsr[k] = ni[k] << (LT - l);
          nzz[k] = TILE >> l;
        }
      }
      wave_sync();
      uint32_t slot[E], q[E];
      bool inner[E];
#pragma unroll
      for (int k = 0; k < E; ++k) {
        const uint32_t p = p0 + k;
        inner[k] = POW2 ? true : (p < s0 && nzz[k] > r);
        slot[k] = sm.Pm[cur][p & (TILE - 1)] & (TILE - 1);
      }
#pragma unroll
      for (int k = 0; k < E; ++k) q[k] = sm.K[d][slot[k]];
      // ---- radix select of each internal node's median code (N << w <= TILE bins);
      // with all codes equal the median is that code and nothing is counted
      if (G > 0) {
        // widest digit with N << w <= TILE bins, at most 8 bits: l + w <=
        // log2(TILE); nodes still split here (two members or more), so l < log2(TILE)
        const uint32_t Wl = umin32(8u, LT - l);
        const uint32_t npass = G <= Wl ? 1u : (G <= 2 * Wl ? 2u : (G + Wl - 1) / Wl);
        const uint32_t firstw = G - (npass - 1) * Wl;
        uint32_t used = 0;
        for (uint32_t pass = 0; pass < npass; ++pass) {
          const uint32_t w = pass == 0 ? firstw : Wl;
          const uint32_t hs = G - used;
          used += w;
          const uint32_t sh = G - used;
          const uint32_t nb = 1u << w, mask = nb - 1;
          if (pass == 0) {
#pragma unroll
            for (int k = 0; k < E; ++k)  // no branch: + 0 outside split nodes
              atomicAdd(&sm.H[(ni[k] << w) + ((q[k] >> sh) & mask)], inner[k] ? 1u : 0u);
          } else {
            uint32_t pre[E];
#pragma unroll
            for (int k = 0; k < E; ++k) pre[k] = sm.npre[ni[k]];
#pragma unroll
            for (int k = 0; k < E; ++k)
              atomicAdd(&sm.H[(ni[k] << w) + ((q[k] >> sh) & mask)],
                        inner[k] && (q[k] >> hs) == pre[k] ? 1u : 0u);  // no branch: + 0
          }
          wave_sync();
          if (N <= 8) {
            // few nodes: every node's bins at once.  The N * 2^w bins are
            // split evenly over the lanes, each lane's bins inside one node;
            // a node's prefix is the wavefront prefix minus its value at the
            // node's first lane.
            const uint32_t T = N << w;
            const uint32_t lp = T > 64 ? bitlen32(T) - 7 : 0u;  // T is a power of two
            const uint32_t per = 1u << lp;                       // bins per lane, <= TILE / 64
            const uint32_t b0 = lane << lp;
            // (b < 64 per <= TILE; bins at or past T were never counted,
            // and leaves' bins only ever got zeros, so every lane reads and
            // clears its bins and at most one lane per node finds the rank,
            // without per-lane branches)
            uint32_t c[TILE / 64];
            uint32_t mine = 0;
#pragma unroll
            for (int k = 0; k < TILE / 64; ++k) {
              const uint32_t b = b0 + k;
              c[k] = (uint32_t)k < per ? sm.H[b] : 0u;
              if ((uint32_t)k < per) sm.H[b] = 0;
              mine += c[k];
            }
            const uint32_t ex = wave_incl(mine) - mine;
            const uint32_t i = b0 < T ? b0 >> w : 0u;
            uint32_t cum = ex - (uint32_t)__shfl((int)ex, (int)((i << w) >> lp));
            const uint32_t rank = sm.nrank[i];
            bool hit = false;
            uint32_t fb = 0, fr = 0;
#pragma unroll
            for (int k = 0; k < TILE / 64; ++k) {
              const bool h = (uint32_t)k < per && cum <= rank && rank < cum + c[k];
              fb = h ? b0 + k : fb;
              fr = h ? rank - cum : fr;
              hit |= h;
              cum += c[k];
            }
            if (hit) {
              sm.npre[i] = (KL)(((uint32_t)sm.npre[i] << w) | (fb & (nb - 1)));
              sm.nrank[i] = (uint16_t)fr;
            }
          } else {  // many small nodes: one lane per node scans its few bins
            for (uint32_t i = lane; i < N; i += 64) {
              if (sm.nsz[i] <= r) continue;
              const uint32_t rank = sm.nrank[i];
              uint32_t cum = 0, found = 0xffffffffu, below = 0;
              for (uint32_t b = 0; b < nb; ++b) {
                const uint32_t c = sm.H[(i << w) + b];
                if (c) sm.H[(i << w) + b] = 0;
                if (found == 0xffffffffu && rank < cum + c) found = b, below = cum;
                cum += c;
              }
              sm.npre[i] = (KL)(((uint32_t)sm.npre[i] << w) | found);
              sm.nrank[i] = (uint16_t)(rank - below);
            }
          }
          wave_sync();
        }
      }
      // ---- stable partition: exclusive prefix of (lt | eq << 16) over the tile
      uint32_t fl[E], jq[E];
      uint32_t mine = 0;
#pragma unroll
      for (int k = 0; k < E; ++k) {
        const uint32_t v = sm.npre[ni[k]];
        jq[k] = sm.nrank[ni[k]];
        fl[k] = inner[k] ? ((q[k] < v ? 1u : 0u) | (q[k] == v ? 0x10000u : 0u)) : 0u;
        mine += fl[k];
      }
      uint32_t ex = wave_incl(mine) - mine;
      // POW2 with nodes of >= E members: the prefix at the lane's node start
      // is the exclusive prefix of the node's first lane
      const bool lane_starts = POW2 && (TILE >> l) >= (uint32_t)E;
      const uint32_t exs = lane_starts ? (uint32_t)__shfl((int)ex, (int)(nsr[0] / E)) : 0u;
      if (!lane_starts) {
        uint32_t e2 = ex;
#pragma unroll
        for (int k = 0; k < E; ++k) {
          if (p0 + k < s0) sm.S[p0 + k] = e2;
          e2 += fl[k];
        }
        wave_sync();
      }
#pragma unroll
      for (int k = 0; k < E; ++k) {
        const uint32_t p = p0 + k;
        const uint32_t ns = nsr[k], nz = nzz[k];
        const uint32_t X = lane_starts ? ex - exs : sm.S[p & (TILE - 1)] - sm.S[ns & (TILE - 1)];
        const uint32_t L = X & 0xffffu, Eq = X >> 16;
        const uint32_t jeq = jq[k];
        const uint32_t lb = L + umin32(Eq, jeq);
        const bool lt = fl[k] & 1u, eq = (fl[k] >> 16) & 1u;
        const bool left = lt || (eq && Eq < jeq);
        const uint32_t dest = inner[k] ? ns + (left ? lb : (nz >> 1) + (p - ns) - lb) : p;
        // every position stores, without a branch: a position past the
        // node's end (or in a leaf) to itself, a member of a split node to
        // its slot, which is below s0 when the counts are right
        sm.Pm[cur ^ 1][dest & (TILE - 1)] = (uint16_t)slot[k];
        ex += fl[k];
        if (!POW2) {  // follow this position into its child of the next level
          const uint32_t half = nz >> 1;
          const bool right = p - ns >= half;
          ni[k] = 2 * ni[k] + (right ? 1u : 0u);
          nsr[k] = right ? ns + half : ns;
          nzz[k] = right ? nz - half : half;
        }
      }
      wave_sync();
      cur ^= 1;
      last_l = (int)l;
      lastN = N;
    }

  };
  if constexpr (TILE == 256 && sizeof(KL) == 2) {  // the first pass at the default capacity
    if (s0 == (uint32_t)TILE && (r & (r - 1)) == 0)
      levels(std::true_type{});
    else
      levels(std::false_type{});
  } else {
    levels(std::false_type{});
  }

  // ---- leaf list (depth-first): nodes of the last level that were split give
  // two leaves, the others are leaves themselves
  uint32_t nl, maxleaf;
  if (last_l < 0) {
    if (lane == 0) sm.H[0] = (uint32_t)s0 << 16;
    nl = 1;
    maxleaf = s0;
  } else {
    const uint32_t N = lastN;
    const uint32_t per = (N + 63) / 64;
    uint32_t cnt = 0;
    for (uint32_t k = 0; k < per; ++k) {
      const uint32_t i = lane * per + k;
      if (i < N) cnt += sm.nsz[i] > r ? 2u : 1u;
    }
    const uint32_t incl = wave_incl(cnt);
    uint32_t at = incl - cnt;
    for (uint32_t k = 0; k < per; ++k) {
      const uint32_t i = lane * per + k;
      if (i >= N) break;
      const uint32_t ns = sm.nst[i], nz = sm.nsz[i];
      if (nz > r) {
        sm.H[at++] = ns | ((nz >> 1) << 16);
        sm.H[at++] = (ns + (nz >> 1)) | ((nz - (nz >> 1)) << 16);
      } else {
        sm.H[at++] = ns | (nz << 16);
      }
    }
    nl = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
    const uint32_t a = s0 / N, b = (s0 + N - 1) / N;  // the two node sizes of the level
    maxleaf = leaf_fold(b, r);
    if (s0 % N != 0 && leaf_fold(a, r) > maxleaf) maxleaf = leaf_fold(a, r);
  }
  wave_sync();

  // ---- bit box per leaf: all leaves in one pass when they fit the wavefront
  // (groups of 64/nl lanes, each lane walking several members), else one lane
  // group per leaf sized to the largest leaf
  uint32_t gs = 1;
  if (nl <= 64) {
    while (gs * 2 * nl <= 64) gs <<= 1;
  }
  while (gs > 1 && gs / 2 >= maxleaf) gs >>= 1;
  const uint32_t span = umax32(Gt[0], umax32(Gt[1], Gt[2]));
  if (TILE == 256 && span <= 14 && maxleaf <= 4 * gs && gs == 8)  // the common shape
    tile_bitboxes<TILE, KL, TRACK, uint32_t, 4, 8>(sm, cur, nl, gs, dims, tmin[0], tmin[1], tmin[2],
                                                   tst, first_leaf, n_leaves, P, leaves, leaf_bits,
                                                   rule);
  else if (TILE == 256 && span <= 14 && maxleaf <= 4 * gs)  // members in registers
    tile_bitboxes<TILE, KL, TRACK, uint32_t, 4>(sm, cur, nl, gs, dims, tmin[0], tmin[1], tmin[2],
                                                tst, first_leaf, n_leaves, P, leaves, leaf_bits,
                                                rule);
  else if (span <= 14)
    tile_bitboxes<TILE, KL, TRACK, uint32_t, 0>(sm, cur, nl, gs, dims, tmin[0], tmin[1], tmin[2],
                                                tst, first_leaf, n_leaves, P, leaves, leaf_bits,
                                                rule);
  else
    tile_bitboxes<TILE, KL, TRACK, uint64_t, 0>(sm, cur, nl, gs, dims, tmin[0], tmin[1], tmin[2],
                                                tst, first_leaf, n_leaves, P, leaves, leaf_bits,
                                                rule);
  wave_sync();

  // ---- write the node back in output-slot order (reference first per leaf)
  for (uint32_t p = lane; p < s0; p += 64) {
    const uint32_t L = sm.S[p];
    const uint32_t ls = sm.H[L] & 0xffffu, ref = sm.lref[L];
    const uint32_t t = p - ls;
    const uint32_t o = t == ref ? 0u : (t < ref ? t + 1 : t);
    const uint32_t slot = sm.Pm[cur][p];
    const uint64_t gpos = tst + ls + o;
#pragma unroll
    for (uint32_t d = 0; d < 3; ++d)
      if (d < dims) keys[(uint64_t)d * kst + gpos] = (KT)(sm.K[d][slot] + tmin[d]);
    if (TRACK && track && perm) perm[gpos] = sm.I[slot];
  }
}

template <int TILE, typename KL, bool TRACK>
__device__ void tile_node(uint32_t nsets, const uint64_t* pre, const SetDesc* sets,
                          DevParams* params, uint8_t* keys0, uint8_t* keys1, uint32_t* idx0,
                          uint32_t* idx1, LeafRec* leaves0, uint64_t* leaf_bits0, uint32_t* defer,
                          uint32_t gtile, WaveTile<TILE, KL, TRACK>& sm) {
  const uint32_t s = find_set(pre, nsets, gtile);
  const SetDesc& S = sets[s];
  DevParams* P = params + s;
  if (P->status != BBX_OK) return;
  const uint64_t j = gtile - pre[s];
  const uint32_t buf = key_buf(S, S.gl);  // the buffer holding the codes at the leaf stage
  uint8_t* keys = (buf ? keys1 : keys0) + S.key_off;
  const uint32_t* idx = S.track ? (buf ? idx1 : idx0) + S.idx_off : nullptr;
  LeafRec* leaves = leaves0 + S.leaf_off;
  uint64_t* leaf_bits = leaf_bits0 + S.leaf_off;
  if (P->key16)
    tile_body<TILE, uint16_t, KL, TRACK>(sm, j, S.gl, S.n, S.kst, S.dims, S.r, S.n_leaves, S.geom,
                                         P, (uint16_t*)keys, idx, S.perm, leaves, leaf_bits, defer,
                                         gtile, S.ref_rule);
  else
    tile_body<TILE, uint32_t, KL, TRACK>(sm, j, S.gl, S.n, S.kst, S.dims, S.r, S.n_leaves, S.geom,
                                         P, (uint32_t*)keys, idx, S.perm, leaves, leaf_bits, defer,
                                         gtile, S.ref_rule);
}

// first pass: every tile, 16-bit tile codes
template <int TILE, bool TRACK>
__global__ void __launch_bounds__(64) k_tile(uint32_t nsets, const uint64_t* pre,
                                             const SetDesc* sets, DevParams* params,
                                             uint8_t* keys0, uint8_t* keys1, uint32_t* idx0,
                                             uint32_t* idx1, LeafRec* leaves0,
                                             uint64_t* leaf_bits0, uint32_t* defer) {
  __shared__ WaveTile<TILE, uint16_t, TRACK> sm;
  tile_node<TILE, uint16_t, TRACK>(nsets, pre, sets, params, keys0, keys1, idx0, idx1, leaves0,
                                   leaf_bits0, defer, blockIdx.x, sm);
}

// second pass: the deferred tiles, 32-bit tile codes (capped grid, striding)
template <int TILE, bool TRACK>
__global__ void __launch_bounds__(64) k_tile_wide(uint32_t nsets, const uint64_t* pre,
                                                  const SetDesc* sets, DevParams* params,
                                                  uint8_t* keys0, uint8_t* keys1, uint32_t* idx0,
                                                  uint32_t* idx1, LeafRec* leaves0,
                                                  uint64_t* leaf_bits0, const uint32_t* defer) {
  __shared__ WaveTile<TILE, uint32_t, TRACK> sm;
  const uint32_t count = defer[0];
  for (uint32_t q = blockIdx.x; q < count; q += gridDim.x) {
    tile_node<TILE, uint32_t, TRACK>(nsets, pre, sets, params, keys0, keys1, idx0, idx1, leaves0,
                                     leaf_bits0, nullptr, defer[1 + q], sm);
    wave_sync();  // the next tile reuses the LDS
  }
}

__global__ void k_zero_u32(uint32_t* p) {
  if (threadIdx.x == 0) *p = 0;
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
__device__ void bigleaf_body(uint64_t i, uint64_t n /* code-array stride */, uint32_t dims,
                             const TreeGeom& g,
                             const KT* src, KT* dst, const uint32_t* idx, uint32_t* perm,
                             LeafRec* leaves, uint64_t* leaf_bits, uint32_t rule) {
  __shared__ uint32_t red[kBlock / 64];
  __shared__ uint64_t rd[kBlock / 64];
  __shared__ uint32_t rp[kBlock / 64];
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
    uint64_t dist;
    if (rule) {  // fewest code bits
      uint32_t bits = 0;
      for (uint32_t d = 0; d < dims; ++d)
        bits += width_of(q[d] - mn[d] > mx[d] - q[d] ? q[d] - mn[d] : mx[d] - q[d]);
      dist = bits;
    } else {  // nearest the AABB centre
      dist = sqdist3(q, C, dims);
    }
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
    rec.ref_src = idx ? idx[st + ref] : 0u;
    leaves[i] = rec;
    leaf_bits[i] = (sz - 1) * (uint64_t)summ;
  }
  for (uint64_t p = threadIdx.x; p < sz; p += kBlock) {
    const uint64_t o = p == ref ? 0 : (p < ref ? p + 1 : p);
    for (uint32_t d = 0; d < dims; ++d) dst[(uint64_t)d * n + st + o] = src[(uint64_t)d * n + st + p];
    if (idx && perm) perm[st + o] = idx[st + p];
  }
}

__global__ void __launch_bounds__(kBlock) k_bigleaf(uint32_t nsets, const uint64_t* pre,
                                                    const SetDesc* sets, DevParams* params,
                                                    uint8_t* keys0, uint8_t* keys1,
                                                    uint32_t* idx0, uint32_t* idx1,
                                                    LeafRec* leaves0, uint64_t* leaf_bits0) {
  const uint32_t s = find_set(pre, nsets, blockIdx.x);
  const SetDesc& S = sets[s];
  DevParams* P = params + s;
  if (P->status != BBX_OK) return;
  const uint32_t buf = key_buf(S, S.gl);  // the buffer holding the codes at the leaf stage
  const uint8_t* src = (buf ? keys1 : keys0) + S.key_off;
  uint8_t* dst = (buf ? keys0 : keys1) + S.key_off;
  const uint32_t* idx = S.track ? (buf ? idx1 : idx0) + S.idx_off : nullptr;
  const uint64_t i = blockIdx.x - pre[s];
  if (P->key16)
    bigleaf_body<uint16_t>(i, S.kst, S.dims, S.geom, (const uint16_t*)src, (uint16_t*)dst, idx,
                           S.perm, leaves0 + S.leaf_off, leaf_bits0 + S.leaf_off, S.ref_rule);
  else
    bigleaf_body<uint32_t>(i, S.kst, S.dims, S.geom, (const uint32_t*)src, (uint32_t*)dst, idx,
                           S.perm, leaves0 + S.leaf_off, leaf_bits0 + S.leaf_off, S.ref_rule);
}

template <int TILE, bool TRACK>
static void launch_tiles(const BatchPlan& bp, const Ws& w, hipStream_t s) {
  BBX_LAUNCH("tile", (k_tile<TILE, TRACK>), bp.g_tile, 64, 0, s, bp.nsets, w.pre + bp.o_tile, w.sets,
             w.params, w.keys[0], w.keys[1], w.idx[0], w.idx[1], w.leaves, w.leaf_bits,
             w.tile_defer);
  const uint64_t gw = bp.g_tile < 4096 ? bp.g_tile : 4096;
  BBX_LAUNCH("tile_wide", (k_tile_wide<TILE, TRACK>), gw, 64, 0, s, bp.nsets, w.pre + bp.o_tile,
             w.sets, w.params, w.keys[0], w.keys[1], w.idx[0], w.idx[1], w.leaves, w.leaf_bits,
             w.tile_defer);
}

hipError_t launch_leaves(const BatchPlan& bp, const Ws& w, hipStream_t s) {
  if (bp.g_tile > 0) {
    BBX_LAUNCH("tile_defer_zero", k_zero_u32, 1, 64, 0, s, w.tile_defer);
    if (bp.tile == 256)
      bp.track ? launch_tiles<256, true>(bp, w, s) : launch_tiles<256, false>(bp, w, s);
    else
      bp.track ? launch_tiles<512, true>(bp, w, s) : launch_tiles<512, false>(bp, w, s);
  }
  if (bp.g_big > 0)
    BBX_LAUNCH("bigleaf", k_bigleaf, bp.g_big, kBlock, 0, s, bp.nsets, w.pre + bp.o_big, w.sets,
               w.params, w.keys[0], w.keys[1], w.idx[0], w.idx[1], w.leaves, w.leaf_bits);
  return hipGetLastError();
}

}  // namespace bbx

// k_reorder.hip -- the two reorderings of Sec. 4.2 applied to the sequence
// layout (bbx_export_sequences) before entropy coding: sequences in
// ascending sum of widths (stable: equal sums keep leaf order), and in each
// sequence the members in ascending R-index, the members' codes concatenated
// with the axes in ascending entropy of their width distributions (first
// axis most significant), equal R-indices in stored order.  A sequence keeps
// its centre, widths and end mark; its members keep their codes.
//
// After the plain export (whose decode leaves every leaf's record and payload
// offset in the decompression workspace):
//   k_ro_hist    per leaf: its widths into per-axis histograms, its key
//                (the sum of widths) and its counts per block of leaves
//   (host: the axis order from the width histograms)
//   k_ro_scan    one block: exclusive scan of the (key, block) counts, key
//                major, so that a key's leaves follow the smaller keys' in
//                block order
//   k_ro_place   per leaf: its place in the new order (its key's base for its
//                block plus the leaves of the block before it with its key);
//                the leaf at each place and that leaf's payload bits there
//   (scan of the placed payload bits: each sequence's new offset)
//   k_ro_write   a wavefront per sequence: centre and widths copied, members
//                ranked by (R-index, stored position), their codes written
//                in that order, the end mark; words ORed into the zeroed
//                output (sequences share boundary words)
#include "bbx_internal.h"

namespace bbx {

typedef unsigned __int128 u128;

constexpr uint32_t kRoKeys = 94;        // sums of widths 0 .. 3 * 31
constexpr uint32_t kRoLocal = 256;      // members ranked from LDS (more: from the layout)
constexpr uint32_t kRoStage = 64;       // words of a sequence staged in LDS (longer: written in place)

__device__ inline uint64_t ro_read(const uint64_t* sec, uint64_t nwords, uint64_t at, uint32_t len) {
  if (len == 0) return 0;
  const uint64_t w = at >> 6;
  const uint32_t s = (uint32_t)(at & 63);
  uint64_t v = w < nwords ? sec[w] >> s : 0ull;
  if (s && s + len > 64 && w + 1 < nwords) v |= sec[w + 1] << (64 - s);
  return len < 64 ? v & ((1ull << len) - 1) : v;
}

__device__ inline void ro_write(unsigned long long* sec, uint64_t at, uint64_t v, uint32_t len) {
  if (len == 0) return;
  if (len < 64) v &= (1ull << len) - 1;
  const uint64_t w = at >> 6;
  const uint32_t s = (uint32_t)(at & 63);
  if (v == 0) return;
  atomicOr(&sec[w], (unsigned long long)(v << s));
  if (s && s + len > 64) atomicOr(&sec[w + 1], (unsigned long long)(v >> (64 - s)));
}

__global__ void __launch_bounds__(kBlock) k_ro_hist(uint64_t n_leaves, uint32_t dims,
                                                    const LeafRec* leaves, uint32_t* whist,
                                                    uint8_t* key, uint32_t* bcount,
                                                    const DevParams* P) {
  if (P->status != BBX_OK) return;
  __shared__ uint32_t kc[kRoKeys];
  __shared__ uint32_t wh[3 * 64];  // the block's width counts, added to the device's once
  for (uint32_t k = threadIdx.x; k < kRoKeys; k += kBlock) kc[k] = 0;
  for (uint32_t k = threadIdx.x; k < 3 * 64; k += kBlock) wh[k] = 0;
  __syncthreads();
  const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n_leaves) {
    const uint32_t m = leaves[i].m;
    uint32_t sm = 0;
    for (uint32_t d = 0; d < dims; ++d) {
      const uint32_t md = (m >> (8 * d)) & 0xffu;
      atomicAdd(&wh[d * 64 + (md & 63)], 1u);
      sm += md;
    }
    key[i] = (uint8_t)sm;
    atomicAdd(&kc[sm < kRoKeys ? sm : kRoKeys - 1], 1u);
  }
  __syncthreads();
  for (uint32_t k = threadIdx.x; k < 3 * 64; k += kBlock)
    if (wh[k]) atomicAdd(&whist[k], wh[k]);
  const uint64_t nblk = gridDim.x;
  for (uint32_t k = threadIdx.x; k < kRoKeys; k += kBlock) bcount[(uint64_t)k * nblk + blockIdx.x] = kc[k];
}

// one block: exclusive scan of counts[key][block], key major
__global__ void __launch_bounds__(1024) k_ro_scan(uint32_t* c, uint64_t entries, const DevParams* P) {
  if (P->status != BBX_OK) return;
  __shared__ uint32_t ws[16];
  uint32_t run = 0;
  for (uint64_t e0 = 0; e0 < entries; e0 += blockDim.x) {
    const uint64_t e = e0 + threadIdx.x;
    const uint32_t v = e < entries ? c[e] : 0u;
    const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint32_t incl = wave_incl(v);
    if (lane == 63) ws[wv] = incl;
    __syncthreads();
    uint32_t off = 0, tot = 0;
    for (uint32_t k = 0; k < blockDim.x / 64; ++k) {
      off += k < wv ? ws[k] : 0u;
      tot += ws[k];
    }
    __syncthreads();
    if (e < entries) c[e] = run + off + incl - v;
    run += tot;
  }
}

__global__ void __launch_bounds__(kBlock) k_ro_place(uint64_t n_leaves, const uint8_t* key,
                                                     const uint32_t* base, const LeafRec* leaves,
                                                     uint32_t* order, uint64_t* sbits,
                                                     const DevParams* P) {
  if (P->status != BBX_OK) return;
  __shared__ uint8_t kl[kBlock];
  const uint64_t i0 = (uint64_t)blockIdx.x * kBlock, i = i0 + threadIdx.x;
  const bool ok = i < n_leaves;
  kl[threadIdx.x] = ok ? key[i] : 0xffu;
  __syncthreads();
  if (!ok) return;
  const uint32_t k = kl[threadIdx.x];
  uint32_t before = 0;
  for (uint32_t t = 0; t < threadIdx.x; ++t) before += kl[t] == k ? 1u : 0u;
  const uint64_t q = base[(uint64_t)k * gridDim.x + blockIdx.x] + before;
  const uint32_t m = leaves[i].m;
  const uint32_t sm = (m & 0xffu) + ((m >> 8) & 0xffu) + ((m >> 16) & 0xffu);
  order[q] = (uint32_t)i;
  sbits[q] = (uint64_t)(leaves[i].size - 1) * sm;
}

__global__ void __launch_bounds__(kBlock) k_ro_zero(uint64_t* p, uint64_t words, const DevParams* P) {
  if (P->status != BBX_OK) return;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < words;
       i += (uint64_t)gridDim.x * kBlock)
    p[i] = 0;
}

// the R-index of member j of a sequence whose codes start at bit `at`
__device__ inline u128 ro_rindex(const uint64_t* pl, uint64_t pw, uint64_t at, uint32_t j,
                                 const uint32_t m[3], uint32_t sm, uint32_t dims, const uint32_t ord[3]) {
  uint64_t u[3] = {0, 0, 0};
  uint64_t p = at + (uint64_t)j * sm;
  for (uint32_t d = 0; d < dims; ++d) {
    u[d] = ro_read(pl, pw, p, m[d]);
    p += m[d];
  }
  u128 r = 0;
  for (uint32_t k = 0; k < dims; ++k) {
    const uint32_t d = ord[k];
    r = (r << m[d]) | (u128)u[d];
  }
  return r;
}

__global__ void __launch_bounds__(kBlock) k_ro_write(uint64_t n_leaves, uint32_t dims, uint32_t M,
                                                     uint32_t mbits, uint32_t o0, uint32_t o1,
                                                     uint32_t o2, const LeafRec* leaves,
                                                     const uint64_t* poff, const uint32_t* order,
                                                     const uint64_t* soff, const uint64_t* plain,
                                                     uint64_t plain_words,
                                                     unsigned long long* out, const DevParams* P) {
  if (P->status != BBX_OK) return;
  __shared__ u128 rk[kBlock / 64][kRoLocal];
  __shared__ unsigned long long stg[kBlock / 64][kRoStage];
  const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint32_t ord[3] = {o0, o1, o2};
  const uint64_t F = (uint64_t)dims * (M + mbits) + 32;  // a sequence's bits besides its codes
  const uint32_t hdr = dims * (M + mbits);
  const uint64_t gw = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  const uint64_t nw = ((uint64_t)gridDim.x * kBlock) >> 6;
  for (uint64_t q = gw; q < n_leaves; q += nw) {
    const uint32_t i = order[q];
    const LeafRec L = leaves[i];
    const uint64_t in = (uint64_t)i * F + poff[i], op = q * F + soff[q];
    const uint32_t m[3] = {L.m & 0xffu, (L.m >> 8) & 0xffu, (L.m >> 16) & 0xffu};
    const uint32_t sm = m[0] + m[1] + m[2];
    const uint32_t cnt = L.size - 1;
    // the sequence's words: staged in LDS when few (then only the two
    // boundary words, shared with the neighbours, need atomics), else ORed
    // into the output in place
    const uint64_t w0 = op >> 6, nwd = ((op + F + (uint64_t)cnt * sm - 1) >> 6) - w0 + 1;
    const bool staged = nwd <= kRoStage;
    unsigned long long* dst = staged ? stg[wv] : out;
    const uint64_t dbase = staged ? w0 * 64 : 0;  // bit offset of dst[0] in the output
    if (staged) {
      for (uint32_t k = lane; k < kRoStage; k += 64) stg[wv][k] = 0;
      wave_sync();
    }
    // centre and widths, 32 bits per lane-step
    for (uint32_t b = lane * 32; b < hdr; b += 64 * 32) {
      const uint32_t c = hdr - b < 32 ? hdr - b : 32;
      ro_write(dst, op + b - dbase, ro_read(plain, plain_words, in + b, c), c);
    }
    const uint64_t cin = in + hdr, cout = op + hdr - dbase;
    if (sm > 0 && cnt > 0) {
      const bool local = cnt <= kRoLocal;
      if (local)
        for (uint32_t j = lane; j < cnt; j += 64)
          rk[wv][j] = ro_rindex(plain, plain_words, cin, j, m, sm, dims, ord);
      wave_sync();
      for (uint32_t j = lane; j < cnt; j += 64) {
        const u128 kj = local ? rk[wv][j] : ro_rindex(plain, plain_words, cin, j, m, sm, dims, ord);
        uint32_t rank = 0;
        for (uint32_t t = 0; t < cnt; ++t) {
          const u128 kt = local ? rk[wv][t] : ro_rindex(plain, plain_words, cin, t, m, sm, dims, ord);
          rank += (kt < kj || (kt == kj && t < j)) ? 1u : 0u;
        }
        // the member's codes, in axis order, at its rank
        uint64_t p = cin + (uint64_t)j * sm, o = cout + (uint64_t)rank * sm;
        for (uint32_t d = 0; d < dims; ++d) {
          ro_write(dst, o, ro_read(plain, plain_words, p, m[d]), m[d]);
          p += m[d];
          o += m[d];
        }
      }
      wave_sync();  // rk is rewritten by the wavefront's next sequence
    }
    if (lane == 0) ro_write(dst, cout + (uint64_t)cnt * sm, 0xffffffffull, 32);  // end mark
    if (staged) {
      wave_sync();
      for (uint32_t k = lane; k < nwd; k += 64) {
        const unsigned long long v = stg[wv][k];
        if (k == 0 || k + 1 == nwd)
          atomicOr(&out[w0 + k], v);
        else
          out[w0 + k] = v;
      }
      wave_sync();  // stg is rewritten by the wavefront's next sequence
    }
  }
}

hipError_t launch_reorder_hist(uint64_t n_leaves, uint32_t dims, const DecompressWs& w,
                               uint32_t* whist, uint8_t* key, uint32_t* bcount, hipStream_t s) {
  const uint64_t nblk = (n_leaves + kBlock - 1) / kBlock;
  if (nblk > 0)
    BBX_LAUNCH("reorder_hist", k_ro_hist, nblk, kBlock, 0, s, n_leaves, dims, w.leaves, whist, key,
               bcount, w.params);
  return hipGetLastError();
}

hipError_t launch_reorder_write(const DecompressPlan& p, const DecompressWs& w, const uint32_t ord[3],
                                const uint8_t* plain, uint8_t* out, uint64_t out_words, uint8_t* key,
                                uint32_t* bcount, uint32_t* order, uint64_t* sbits, hipStream_t s) {
  const uint64_t nl = p.n_leaves, nblk = (nl + kBlock - 1) / kBlock;
  if (nl == 0) return hipGetLastError();
  const uint32_t M = coord_bits(p.dtype);
  BBX_LAUNCH("reorder_scan", k_ro_scan, 1, 1024, 0, s, bcount, (uint64_t)kRoKeys * nblk, w.params);
  BBX_LAUNCH("reorder_place", k_ro_place, nblk, kBlock, 0, s, nl, key, bcount, w.leaves, order, sbits,
             w.params);
  hipError_t e = launch_dec_scan(nl, sbits, w.scan_part, w.params, p.payload_bits, s);
  if (e != hipSuccess) return e;
  BBX_LAUNCH("reorder_zero", k_ro_zero, (uint32_t)std::min<uint64_t>(out_words / kBlock + 1, 4096), kBlock, 0,
             s, (uint64_t*)out, out_words, w.params);
  const uint64_t plain_words = out_words;  // both layouts have the same length
  BBX_LAUNCH("reorder_write", k_ro_write, (uint32_t)std::min<uint64_t>((nl + 3) / 4, 65536), kBlock, 0, s,
             nl, p.dims, M, p.mbits, ord[0], ord[1], ord[2], w.leaves, w.leaf_bits, order, sbits,
             (const uint64_t*)plain, plain_words, (unsigned long long*)out, w.params);
  return hipGetLastError();
}

}  // namespace bbx

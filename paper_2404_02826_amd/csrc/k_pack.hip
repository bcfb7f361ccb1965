// k_pack.hip -- leaf bit offsets and bit packing (Sec. 4.2, storage layout),
// for every set of a batch.
//
//   k_scan_reduce / k_scan_top / k_scan_down
//        exclusive prefix sum of the per-leaf payload bits over the whole
//        batch (depth-first leaf order inside each set); a set's offsets are
//        differences against its first leaf's offset
//   k_set_sizes     per set: payload and meta bits, stream size, capacity check
//   k_pack_meta     one thread per 64-bit meta word: gathers the fixed-stride
//                   leaf records (widths, reference codes) that overlap it
//   k_pack_payload  leaf-aligned blocks: each block owns the payload words
//                   that start inside its leaves, ORs every member code
//                   q - q_ref + 2^(m-1) into an LDS copy of those words (LDS
//                   atomics; 8 consecutive members per thread, assembled in
//                   registers and ORed a word at a time when they share a
//                   leaf), completes its last word from the next leaves (a
//                   member per lane), then writes every owned word once with
//                   a coalesced plain store (no global atomics, no zeroing of
//                   the output)
//   k_header        the 128-byte header
//   k_finish        reports size and status
#include "bbx_internal.h"

namespace bbx {

typedef unsigned __int128 u128;

constexpr int kScanPer = 16;
constexpr uint64_t kScanChunk = (uint64_t)kBlock * kScanPer;

uint64_t scan_blocks(uint64_t count) { return (count + kScanChunk - 1) / kScanChunk; }

__device__ inline uint64_t bexscan(uint64_t v, uint64_t* total) {
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

// P (optional): skip when its status is not OK
__global__ void __launch_bounds__(kBlock) k_scan_reduce(uint64_t count, const uint64_t* bits,
                                                        uint64_t* part, const DevParams* P) {
  if (P && P->status != BBX_OK) return;
  const uint64_t base = blockIdx.x * kScanChunk + (uint64_t)threadIdx.x * kScanPer;
  uint64_t s = 0;
  for (int k = 0; k < kScanPer; ++k)
    if (base + k < count) s += bits[base + k];
  uint64_t tot;
  (void)bexscan(s, &tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// Exclusive scan of the block partials; the grand total goes to *total.
// With P: the total must equal expect (decoding) or the status turns ECORRUPT.
__global__ void __launch_bounds__(kBlock) k_scan_top(uint64_t nparts, uint64_t* part,
                                                     uint64_t* total, DevParams* P,
                                                     uint64_t expect) {
  if (P && P->status != BBX_OK) return;
  const uint64_t per = (nparts + kBlock - 1) / kBlock;
  const uint64_t b0 = threadIdx.x * per;
  uint64_t s = 0;
  for (uint64_t k = 0; k < per; ++k)
    if (b0 + k < nparts) s += part[b0 + k];
  uint64_t tot;
  uint64_t run = bexscan(s, &tot);
  for (uint64_t k = 0; k < per; ++k)
    if (b0 + k < nparts) {
      const uint64_t v = part[b0 + k];
      part[b0 + k] = run;
      run += v;
    }
  if (threadIdx.x == 0) {
    if (total) *total = tot;
    if (P) {
      if (tot != expect) P->status = BBX_ECORRUPT;
      P->payload_bits = tot;
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_scan_down(uint64_t count, uint64_t* bits,
                                                      const uint64_t* part, const DevParams* P) {
  if (P && P->status != BBX_OK) return;
  const uint64_t base = blockIdx.x * kScanChunk + (uint64_t)threadIdx.x * kScanPer;
  uint64_t v[kScanPer];
  uint64_t s = 0;
  for (int k = 0; k < kScanPer; ++k) {
    v[k] = base + k < count ? bits[base + k] : 0;
    s += v[k];
  }
  uint64_t tot;
  uint64_t run = bexscan(s, &tot) + part[blockIdx.x];
  for (int k = 0; k < kScanPer; ++k)
    if (base + k < count) {
      bits[base + k] = run;
      run += v[k];
    }
}

static hipError_t scan_launch(uint64_t count, uint64_t* bits, uint64_t* part, uint64_t* total,
                              DevParams* P, uint64_t expect, hipStream_t s) {
  const uint64_t nb = scan_blocks(count);
  if (nb > 0) BBX_LAUNCH("scan_reduce", k_scan_reduce, nb, kBlock, 0, s, count, bits, part, P);
  BBX_LAUNCH("scan_top", k_scan_top, 1, kBlock, 0, s, nb, part, total, P, expect);
  if (nb > 0) BBX_LAUNCH("scan_down", k_scan_down, nb, kBlock, 0, s, count, bits, part, P);
  return hipGetLastError();
}

hipError_t launch_dec_scan(uint64_t count, uint64_t* bits, uint64_t* part, DevParams* params,
                           uint64_t expect_payload, hipStream_t s) {
  return scan_launch(count, bits, part, nullptr, params, expect_payload, s);
}

// per set: payload/meta bits, stream size, capacity check
__global__ void k_set_sizes(uint32_t nsets, const SetDesc* sets, DevParams* params,
                            const uint64_t* off, uint64_t total_leaves, const uint64_t* total,
                            uint32_t* lossless) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsets) return;
  const SetDesc& S = sets[s];
  DevParams* P = params + s;
  if (P->status == kStatusLossless) {  // every coordinate as its bits, no meta section
    P->payload_base = 0;
    P->meta_bits = 0;
    P->payload_bits = S.n * S.dims * coord_bits(S.dtype);
    P->total_bytes = kHeaderBytes + ((P->payload_bits + 63) / 64) * 8;
    if (P->total_bytes > S.out_cap)
      P->status = BBX_ENOSPC;
    else
      lossless[1 + atomicAdd(lossless, 1u)] = s;  // for k_lossless
    return;
  }
  if (P->status != BBX_OK) return;
  const uint64_t b = S.leaf_off, e = S.leaf_off + S.n_leaves;
  const uint64_t base = S.n_leaves ? off[b] : 0;
  const uint64_t endv = S.n_leaves ? (e < total_leaves ? off[e] : *total) : 0;
  uint32_t sumG = 0;  // reference field: codes, or original coordinates with ref_mode 1
  for (uint32_t d = 0; d < S.dims; ++d) sumG += S.ref_mode ? coord_bits(S.dtype) : P->G[d];
  // one record per leaf; with the bit box reduction one per sequence, with
  // a 32-bit particle count
  const uint64_t meta = seq_stream(S) ? P->nseq * (uint64_t)(S.dims * S.mbits + sumG + 32)
                                 : S.n_leaves * (uint64_t)(S.dims * S.mbits + sumG);
  P->payload_base = base;
  P->meta_bits = meta;
  P->payload_bits = endv - base;
  P->total_bytes = kHeaderBytes + ((meta + 63) / 64) * 8 + ((P->payload_bits + 63) / 64) * 8;
  if (P->total_bytes > S.out_cap) P->status = BBX_ENOSPC;
}

// ---------------------------------------------------------------- packing

// OR the bits of `val` (len bits, whose bit 0 sits at absolute bit `at`) into
// the 64-bit word whose bit 0 sits at absolute bit `w0`.
__device__ inline void or_into(uint64_t& word, uint64_t w0, u128 val, uint64_t at, uint32_t len) {
  if (len == 0) return;
  const int64_t rel = (int64_t)(at - w0);
  if (rel >= 64 || rel + (int64_t)len <= 0) return;
  if (len < 128) val &= (((u128)1) << len) - 1;
  if (rel >= 0)
    word |= (uint64_t)(val << rel);
  else
    word |= (uint64_t)(val >> (-rel));
}

// Bits of the reference's original coordinate on axis d (ref_mode 1): the
// caller's value at the reference's source index.
__device__ inline uint64_t ref_coord_bits(const SetDesc& S, uint32_t src, uint32_t d) {
  const uint64_t k = S.layout == BBX_AOS ? (uint64_t)src * S.dims + d : (uint64_t)d * S.n + src;
  if (S.dtype == BBX_F32) return ((const uint32_t*)S.pos)[k];
  return ((const uint64_t*)S.pos)[k];
}

__global__ void __launch_bounds__(kBlock) k_pack_meta(uint32_t nsets, const uint64_t* pre,
                                                      const SetDesc* sets,
                                                      const DevParams* params,
                                                      const LeafRec* leaves0) {
  const uint32_t s = find_set(pre, nsets, blockIdx.x);
  const SetDesc& S = sets[s];
  const DevParams* P = params + s;
  if (P->status != BBX_OK) return;
  const uint64_t lb = blockIdx.x - pre[s], nblk = pre[s + 1] - pre[s];
  const uint32_t dims = S.dims, mbits = S.mbits;
  const uint32_t G[3] = {P->G[0], P->G[1], P->G[2]};
  const uint64_t nwords = (P->meta_bits + 63) / 64;
  const LeafRec* leaves = leaves0 + S.leaf_off;
  uint64_t* meta = (uint64_t*)(S.out + kHeaderBytes);
  if (S.ref_mode) {  // records of dims * (mbits + M) bits, written field by field
    const uint32_t M = coord_bits(S.dtype);
    const uint32_t Sb = dims * (mbits + M);
    for (uint64_t w = lb * blockDim.x + threadIdx.x; w < nwords; w += nblk * blockDim.x) {
      const uint64_t b0 = w * 64;
      const uint64_t i0 = b0 / Sb;
      uint64_t i1 = (b0 + 63) / Sb;
      if (i1 >= S.n_leaves) i1 = S.n_leaves - 1;
      uint64_t word = 0;
      for (uint64_t i = i0; i <= i1; ++i) {
        const LeafRec rec = leaves[i];
        uint64_t at = i * Sb;
        for (uint32_t d = 0; d < dims; ++d, at += mbits)
          or_into(word, b0, (rec.m >> (8 * d)) & 0xffu, at, mbits);
        for (uint32_t d = 0; d < dims; ++d, at += M)
          or_into(word, b0, ref_coord_bits(S, rec.ref_src, d), at, M);
      }
      meta[w] = word;
    }
    return;
  }
  uint32_t Sb = dims * mbits;
  for (uint32_t d = 0; d < dims; ++d) Sb += G[d];
  for (uint64_t w = lb * blockDim.x + threadIdx.x; w < nwords; w += nblk * blockDim.x) {
    const uint64_t b0 = w * 64;
    const uint64_t i0 = b0 / Sb;
    uint64_t i1 = (b0 + 63) / Sb;
    if (i1 >= S.n_leaves) i1 = S.n_leaves - 1;
    uint64_t word = 0;
    for (uint64_t i = i0; i <= i1; ++i) {
      const LeafRec rec = leaves[i];
      u128 v = 0;
      uint32_t at = 0;
      for (uint32_t d = 0; d < dims; ++d) {
        v |= (u128)((rec.m >> (8 * d)) & 0xffu) << at;
        at += mbits;
      }
      for (uint32_t d = 0; d < dims; ++d) {
        v |= (u128)rec.qref[d] << at;
        at += G[d];
      }
      or_into(word, b0, v, i * Sb, Sb);
    }
    meta[w] = word;
  }
}

template <typename KT>
__device__ inline u128 member_code(const KT* keys, uint64_t stride, uint32_t dims, const LeafRec& rec,
                                   uint64_t slot) {
  u128 v = 0;
  uint32_t at = 0;
#pragma unroll
  for (uint32_t d = 0; d < 3; ++d) {
    if (d >= dims) break;
    const uint32_t m = (rec.m >> (8 * d)) & 0xffu;
    if (m == 0) continue;
    const uint32_t q = keys[(uint64_t)d * stride + slot];
    const uint64_t u = (uint64_t)((int64_t)q - (int64_t)rec.qref[d] + ((int64_t)1 << (m - 1)));
    v |= (u128)u << at;
    at += m;
  }
  return v;
}

__device__ inline uint32_t sum_m(uint32_t m) { return (m & 0xffu) + ((m >> 8) & 0xffu) + ((m >> 16) & 0xffu); }

// largest i in [lo, hi] with off[i] - base <= b (offsets non-decreasing)
__device__ inline uint64_t search_off(const uint64_t* off, uint64_t base, uint64_t lo, uint64_t hi,
                                      uint64_t b) {
  while (lo < hi) {
    const uint64_t mid = lo + (hi - lo + 1) / 2;
    if (off[mid] - base <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

constexpr uint32_t kLeafStage = 256;   // leaves per block (leaves_per_block)

// 64-bit forms for members whose code has at most 64 bits (the usual case)
template <typename KT>
__device__ inline uint64_t member_code64(const KT* base, uint64_t stride, uint32_t dims,
                                         const LeafRec& rec, uint64_t t) {
  uint64_t v = 0;
  uint32_t at = 0;
#pragma unroll
  for (uint32_t d = 0; d < 3; ++d) {
    if (d >= dims) break;
    const uint32_t m = (rec.m >> (8 * d)) & 0xffu;
    if (m == 0) continue;
    const uint32_t q = base[d * stride + t];
    const uint64_t u = (uint64_t)((int64_t)q - (int64_t)rec.qref[d] + ((int64_t)1 << (m - 1)));
    v |= u << at;
    at += m;
  }
  return v;
}
// OR a code of len <= 64 bits starting at absolute bit `at` into the word at w0
__device__ inline void or_into64(uint64_t& word, uint64_t w0, uint64_t val, uint64_t at) {
  if (at >= w0)
    word |= val << (uint32_t)(at - w0);  // at - w0 < 64 (callers keep at < w0 + 64)
  else
    word |= val >> (uint32_t)(w0 - at);  // w0 - at < len <= 64
}

constexpr uint32_t kPackLdsWords = 3072;  // payload words of one block's members (24 KB)

// Leaf-aligned packing: a block takes leaves_per_block(r) consecutive leaves
// and stages their records and bit offsets.  Every member (thread per slot,
// coalesced code loads) ORs its code into an LDS copy of the payload words its
// leaves' bits touch (LDS atomics), and the block stores the words whose first
// bit lies in its leaves' bit range with coalesced plain stores.  The last such
// word can also hold the first bits of the next block's leaves: one thread
// adds those few members from global memory.  Blocks whose bits exceed the LDS
// copy (very large leaves) assemble each word from global memory instead.
template <typename KT>
__device__ void pack_payload_body(const SetDesc& S, const DevParams* P, uint64_t blk,
                                  const LeafRec* leaves, const uint64_t* off, const KT* keys,
                                  LeafRec* s_rec, uint64_t* s_off, unsigned long long* s_w) {
  const uint64_t kst = S.kst, nl = S.n_leaves, base = P->payload_base, pbits = P->payload_bits;
  const uint32_t dims = S.dims;
  const uint32_t lpb = leaves_per_block(S.r);
  const uint64_t L0 = blk * lpb;
  if (L0 >= nl) return;
  const uint32_t nlb = (uint32_t)(nl - L0 < lpb ? nl - L0 : lpb);
  for (uint32_t t = threadIdx.x; t < nlb; t += kBlock) {
    s_rec[t] = leaves[L0 + t];
    s_off[t] = off[L0 + t] - base;
  }
  const uint64_t bo1 = L0 + nlb < nl ? off[L0 + nlb] - base : pbits;
  __syncthreads();
  const uint64_t bo0 = s_off[0];
  if (bo1 <= bo0) return;  // no payload bits in these leaves (uniform)
  uint64_t* pay = (uint64_t*)(S.out + kHeaderBytes + ((P->meta_bits + 63) / 64) * 8);
  const uint64_t w_first = (bo0 + 63) / 64, w_end = (bo1 + 63) / 64;  // owned words
  const uint64_t wlo = bo0 / 64;
  const uint64_t nwb = w_end - wlo;
  const uint64_t Lend = L0 + nlb;
  if (nwb > kPackLdsWords) {  // large leaves: each owned word from global memory
    for (uint64_t w = w_first + threadIdx.x; w < w_end; w += kBlock) {
      const uint64_t b0 = w * 64;
      uint32_t a = 0, z = nlb - 1;
      while (a < z) {
        const uint32_t mid = (a + z + 1) >> 1;
        if (s_off[mid] <= b0)
          a = mid;
        else
          z = mid - 1;
      }
      uint64_t i = L0 + a;
      LeafRec rec = s_rec[a];
      uint32_t sm = sum_m(rec.m);
      const uint64_t oi = s_off[a];
      uint64_t jm = sm ? (b0 - oi) / sm : 0;
      uint64_t at = oi + jm * sm;
      uint64_t word = 0;
      while (at < b0 + 64) {
        if (sm > 0 && jm + 1 < rec.size) {
          const u128 c = member_code(keys, kst, dims, rec, (uint64_t)rec.start + 1 + jm);
          or_into(word, b0, c, at, sm);
          at += sm;
          ++jm;
        } else {
          ++i;
          if (i >= nl) break;
          rec = i < Lend ? s_rec[i - L0] : leaves[i];
          sm = sum_m(rec.m);
          jm = 0;
        }
      }
      pay[w] = word;
    }
    return;
  }
  for (uint32_t t = threadIdx.x; t < (uint32_t)nwb; t += kBlock) s_w[t] = 0;
  __syncthreads();
  const uint64_t slot0 = s_rec[0].start;
  const uint64_t slot_end = (uint64_t)s_rec[nlb - 1].start + s_rec[nlb - 1].size;
  // each thread takes V consecutive slots (V-aligned slot indices): one
  // 16-byte code load per axis, one leaf search, and LDS atomics that land on
  // different words across the lanes
  constexpr uint32_t V = 16 / sizeof(KT);
  for (uint64_t gs = (slot0 & ~(uint64_t)(V - 1)) + (uint64_t)V * threadIdx.x; gs < slot_end;
       gs += (uint64_t)V * kBlock) {
    union {
      uint4 v;
      KT e[V];
    } kk[3];
#pragma unroll
    for (uint32_t d = 0; d < 3; ++d) {
      kk[d].v = make_uint4(0, 0, 0, 0);
      if (d < dims) kk[d].v = *(const uint4*)(keys + (uint64_t)d * kst + gs);
    }
    const uint64_t pfirst = gs > slot0 ? gs : slot0;
    uint32_t a = 0, z = nlb - 1;  // last staged leaf starting at or before pfirst
    while (a < z) {
      const uint32_t mid = (a + z + 1) >> 1;
      if (s_rec[mid].start <= pfirst)
        a = mid;
      else
        z = mid - 1;
    }
    {
      // the usual shape: all V slots inside leaf a, member codes of at most
      // 32 bits.  The run's codes occupy consecutive bits, so they are
      // assembled in registers and ORed into LDS one 64-bit word at a time.
      const LeafRec ra = s_rec[a];
      const uint32_t sma = sum_m(ra.m);
      if (gs >= ra.start && gs + V <= (uint64_t)ra.start + ra.size && sma > 0 && sma <= 32) {
        const uint32_t j0 = (uint32_t)(gs - ra.start);
        uint32_t hm[3], sh3[3] = {0, 0, 0};
#pragma unroll
        for (uint32_t d = 0; d < 3; ++d) {
          const uint32_t m = d < dims ? (ra.m >> (8 * d)) & 0xffu : 0u;
          hm[d] = (uint32_t)((1ull << m) >> 1) - (d < dims ? ra.qref[d] : 0u);
          if (d + 1 < 3) sh3[d + 1] = sh3[d] + m;
        }
        uint32_t at = (uint32_t)(s_off[a] - wlo * 64) + (j0 ? j0 - 1 : 0u) * sma;
        uint32_t w = at >> 6, pos = at & 63;
        uint64_t lo = 0, hi = 0;
#pragma unroll
        for (uint32_t k = 0; k < V; ++k) {
          if (j0 + k == 0) continue;  // the reference carries no payload
          uint64_t c = 0;
#pragma unroll
          for (uint32_t d = 0; d < 3; ++d)
            if (d < dims) c |= (uint64_t)((uint32_t)kk[d].e[k] + hm[d]) << sh3[d];
          lo |= c << pos;
          hi |= pos ? c >> (64 - pos) : 0ull;
          pos += sma;
          if (pos >= 64) {
            atomicOr(&s_w[w], (unsigned long long)lo);
            ++w;
            lo = hi;
            hi = 0;
            pos -= 64;
          }
        }
        if (pos > 0) atomicOr(&s_w[w], (unsigned long long)lo);
        continue;
      }
    }
#pragma unroll
    for (uint32_t k = 0; k < V; ++k) {
      const uint64_t slot = gs + k;
      if (slot < slot0 || slot >= slot_end) continue;
      while (a + 1 < nlb && s_rec[a + 1].start <= slot) ++a;
      const LeafRec rec = s_rec[a];
      const uint32_t j = (uint32_t)(slot - rec.start);
      const uint32_t sm = sum_m(rec.m);
      if (j == 0 || sm == 0) continue;  // the reference, or a leaf without payload
      // bit in the LDS copy (below kPackLdsWords * 64: 32-bit arithmetic)
      const uint32_t at = (uint32_t)(s_off[a] - wlo * 64) + (j - 1) * sm;
      const uint32_t w = at >> 6, sh = at & 63;
      if (sm <= 64) {
        // u_d = q_d - q_ref,d + 2^(m_d - 1) lies in [0, 2^m_d) (m_d <= 32), so
        // 32-bit wrap-around arithmetic gives it exactly; an axis with m_d = 0
        // has q_d = q_ref,d and adds nothing
        uint64_t c = 0;
        uint32_t cat = 0;
#pragma unroll
        for (uint32_t d = 0; d < 3; ++d) {
          if (d >= dims) break;
          const uint32_t m = (rec.m >> (8 * d)) & 0xffu;
          const uint32_t u = (uint32_t)kk[d].e[k] - rec.qref[d] + (uint32_t)((1ull << m) >> 1);
          c |= (uint64_t)u << cat;
          cat += m;
        }
        atomicOr(&s_w[w], (unsigned long long)(c << sh));
        if (sh + sm > 64) atomicOr(&s_w[w + 1], (unsigned long long)(c >> (64 - sh)));
      } else {
        const u128 c = member_code(keys, kst, dims, rec, slot) << sh;
        atomicOr(&s_w[w], (unsigned long long)(uint64_t)c);
        atomicOr(&s_w[w + 1], (unsigned long long)(uint64_t)(c >> 64));
        if (sh + sm > 128) {
          const u128 c3 = member_code(keys, kst, dims, rec, slot) >> (128 - sh);
          atomicOr(&s_w[w + 2], (unsigned long long)(uint64_t)c3);
        }
      }
    }
  }
  __syncthreads();
  if ((bo1 & 63) != 0 && bo1 < pbits && threadIdx.x < 64) {
    // bits [bo1, w_end * 64) of the last owned word come from the next leaves
    // (bo1 < pbits: leaf Lend exists).  When leaf Lend alone holds them, the
    // first wavefront adds one member per lane; otherwise one thread walks
    // the following leaves.
    const uint64_t b0 = (w_end - 1) * 64, need = w_end * 64 - bo1;
    const LeafRec rn = leaves[Lend];
    const uint32_t smn = sum_m(rn.m);
    if (smn > 0 && (uint64_t)(rn.size - 1) * smn >= need) {
      const uint32_t t = threadIdx.x;
      const uint64_t at = bo1 + (uint64_t)t * smn;
      if (t + 1 < rn.size && at < w_end * 64) {
        uint64_t part = 0;
        or_into(part, b0, member_code(keys, kst, dims, rn, (uint64_t)rn.start + 1 + t), at, smn);
        atomicOr(&s_w[w_end - 1 - wlo], (unsigned long long)part);
      }
    } else if (threadIdx.x == 0) {
      uint64_t word = s_w[w_end - 1 - wlo];
      uint64_t i = Lend;
      uint64_t at = bo1;
      while (i < nl && at < w_end * 64) {
        const LeafRec rec = leaves[i];
        const uint32_t sm = sum_m(rec.m);
        for (uint64_t jm = 0; sm > 0 && jm + 1 < rec.size && at < w_end * 64; ++jm) {
          const u128 c = member_code(keys, kst, dims, rec, (uint64_t)rec.start + 1 + jm);
          or_into(word, b0, c, at, sm);
          at += sm;
        }
        ++i;
      }
      s_w[w_end - 1 - wlo] = word;
    }
  }
  __syncthreads();
  for (uint64_t w = w_first + threadIdx.x; w < w_end; w += kBlock) pay[w] = s_w[w - wlo];
}

__global__ void __launch_bounds__(kBlock) k_pack_payload(uint32_t nsets, const uint64_t* pre,
                                                         const SetDesc* sets,
                                                         const DevParams* params,
                                                         const LeafRec* leaves0,
                                                         const uint64_t* off0,
                                                         const uint8_t* keys0,
                                                         const uint8_t* keys1) {
  const uint32_t s = find_set(pre, nsets, blockIdx.x);
  const SetDesc& S = sets[s];
  const DevParams* P = params + s;
  if (P->status != BBX_OK) return;
  if (P->payload_bits == 0) return;
  __shared__ LeafRec s_rec[kLeafStage];
  __shared__ uint64_t s_off[kLeafStage];
  __shared__ unsigned long long s_w[kPackLdsWords];
  const uint64_t blk = blockIdx.x - pre[s];
  const uint8_t* keys = (S.final_buf ? keys1 : keys0) + S.key_off;
  const LeafRec* leaves = leaves0 + S.leaf_off;
  const uint64_t* off = off0 + S.leaf_off;
  if (P->key16)
    pack_payload_body<uint16_t>(S, P, blk, leaves, off, (const uint16_t*)keys, s_rec, s_off, s_w);
  else
    pack_payload_body<uint32_t>(S, P, blk, leaves, off, (const uint32_t*)keys, s_rec, s_off, s_w);
}

__global__ void k_header(const SetDesc* sets, const DevParams* params) {
  const SetDesc& S = sets[blockIdx.x];
  const DevParams* P = params + blockIdx.x;
  const bool lossless = P->status == kStatusLossless;
  if (P->status != BBX_OK && !lossless) return;
  if (threadIdx.x != 0) return;
  const uint32_t dims = S.dims;
  uint64_t h[16];
  for (int k = 0; k < 16; ++k) h[k] = 0;
  const uint64_t ver = lossless ? 3 : (seq_stream(S) ? 2 : 1);
  h[0] = (uint64_t)kMagic | (ver << 32) | ((uint64_t)S.dtype << 48) | ((uint64_t)dims << 56);
  if (lossless) {  // no grid, no leaves, no meta section; no reference field
    h[1] = S.n;
    h[2] = (uint64_t)S.r | ((uint64_t)S.eb_mode << 32) | ((uint64_t)S.mbits << 56);
    h[3] = __double_as_longlong(P->eb_user);
    h[4] = __double_as_longlong(P->eb_abs);
    h[14] = P->payload_bits;
    uint64_t* o = (uint64_t*)S.out;
    for (int k = 0; k < 16; ++k) o[k] = h[k];
    return;
  }
  h[1] = S.n;
  h[2] = (uint64_t)S.r | ((uint64_t)S.eb_mode << 32) | ((uint64_t)S.split << 40) |
         ((uint64_t)S.ref_mode << 48) | ((uint64_t)S.mbits << 56);
  h[3] = __double_as_longlong(P->eb_user);
  h[4] = __double_as_longlong(P->eb_abs);
  h[5] = __double_as_longlong(P->eb_eff);
  h[6] = __double_as_longlong(P->w);
  h[7] = __double_as_longlong(P->inv_w);
  for (uint32_t d = 0; d < 3; ++d) h[8 + d] = d < dims ? __double_as_longlong(P->lo[d]) : 0;
  h[11] = (uint64_t)P->G[0] | ((uint64_t)(dims > 1 ? P->G[1] : 0) << 8) |
          ((uint64_t)(dims > 2 ? P->G[2] : 0) << 16);
  h[12] = S.split ? P->nleaves : S.n_leaves;  // a split-rule partition's count is the device's
  h[13] = P->meta_bits;
  h[14] = P->payload_bits;
  h[15] = seq_stream(S) ? P->nseq : 0;  // version 2: the sequence count
  uint64_t* o = (uint64_t*)S.out;
  for (int k = 0; k < 16; ++k) o[k] = h[k];
}

__global__ void k_finish(uint32_t nsets, const SetDesc* sets, const DevParams* params) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsets) return;
  const SetDesc& S = sets[s];
  const uint32_t st = params[s].status == kStatusLossless ? BBX_OK : params[s].status;
  if (S.d_size) *S.d_size = st == BBX_OK ? params[s].total_bytes : ~0ull;
  if (S.d_status) *S.d_status = st;
}

__device__ void lossless_copy(const SetDesc& S, uint64_t lb, uint64_t nblk) {
  const uint64_t nv = S.n * S.dims, step = nblk * kBlock;
  uint8_t* pay = S.out + kHeaderBytes;
  if (S.dtype == BBX_F32) {
    const uint32_t* in = (const uint32_t*)S.pos;
    uint32_t* out = (uint32_t*)pay;
    for (uint64_t k = lb * kBlock + threadIdx.x; k < nv; k += step) {
      const uint64_t i = k / S.dims, d = k - i * S.dims;
      out[k] = S.layout == BBX_AOS ? in[k] : in[d * S.n + i];
    }
    if (lb == 0 && threadIdx.x == 0 && (nv & 1)) out[nv] = 0;  // zero padding to 8 bytes
  } else {
    const uint64_t* in = (const uint64_t*)S.pos;
    uint64_t* out = (uint64_t*)pay;
    for (uint64_t k = lb * kBlock + threadIdx.x; k < nv; k += step) {
      const uint64_t i = k / S.dims, d = k - i * S.dims;
      out[k] = S.layout == BBX_AOS ? in[k] : in[d * S.n + i];
    }
  }
  uint32_t* perm = seq_stream(S) ? S.user_perm : S.perm;
  if (perm)
    for (uint64_t i = lb * kBlock + threadIdx.x; i < S.n; i += step) perm[i] = (uint32_t)i;
}

// The sets stored losslessly (listed by k_set_sizes): their coordinates'
// bits, particle by particle in input order (x, y, z), M bits each,
// zero-padded to 8 bytes; perm is the identity.  A fixed grid shares each
// listed set's copy; with no such set every block exits at once.
constexpr uint32_t kLosslessBlocks = 256;
__global__ void __launch_bounds__(kBlock) k_lossless(const SetDesc* sets, const uint32_t* list) {
  const uint32_t count = list[0];
  for (uint32_t li = 0; li < count; ++li) {
    const SetDesc& S = sets[list[1 + li]];
    lossless_copy(S, blockIdx.x, kLosslessBlocks);
  }
}

hipError_t launch_pack(const BatchPlan& bp, const Ws& w, hipStream_t s) {
  hipError_t e = scan_launch(bp.total_leaves, w.leaf_bits, w.scan_part, w.scan_total, nullptr, 0, s);
  if (e != hipSuccess) return e;
  const uint32_t g = (bp.nsets + kBlock - 1) / kBlock;
  BBX_LAUNCH("set_sizes", k_set_sizes, g, kBlock, 0, s, bp.nsets, w.sets, w.params, w.leaf_bits,
             bp.total_leaves, w.scan_total, w.lossless);
  if (bp.g_pm > 0)
    BBX_LAUNCH("pack_meta", k_pack_meta, bp.g_pm, kBlock, 0, s, bp.nsets, w.pre + bp.o_pm, w.sets,
               w.params, w.leaves);
  if (bp.g_pp > 0)
    BBX_LAUNCH("pack_payload", k_pack_payload, bp.g_pp, kBlock, 0, s, bp.nsets, w.pre + bp.o_pp,
               w.sets, w.params, w.leaves, w.leaf_bits, w.keys[0], w.keys[1]);
  e = launch_reduce_pack(bp, w, s);
  if (e != hipSuccess) return e;
  BBX_LAUNCH("lossless", k_lossless, kLosslessBlocks, kBlock, 0, s, w.sets, w.lossless);
  BBX_LAUNCH("header", k_header, bp.nsets, 64, 0, s, w.sets, w.params);
  BBX_LAUNCH("finish", k_finish, g, kBlock, 0, s, bp.nsets, w.sets, w.params);
  return hipGetLastError();
}

}  // namespace bbx

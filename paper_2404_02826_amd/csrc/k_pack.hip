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
//   k_pack_payload  one thread per 64-bit payload word: finds the leaf holding
//                   the word's first bit and gathers the member codes
//                   q - q_ref + 2^(m-1) that overlap it, so every word is
//                   written once with a plain store (no atomics, no zeroing)
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
                            const uint64_t* off, uint64_t total_leaves, const uint64_t* total) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsets) return;
  const SetDesc& S = sets[s];
  DevParams* P = params + s;
  if (P->status != BBX_OK) return;
  const uint64_t b = S.leaf_off, e = S.leaf_off + S.n_leaves;
  const uint64_t base = S.n_leaves ? off[b] : 0;
  const uint64_t endv = S.n_leaves ? (e < total_leaves ? off[e] : *total) : 0;
  uint32_t sumG = 0;
  for (uint32_t d = 0; d < S.dims; ++d) sumG += P->G[d];
  const uint64_t meta = S.n_leaves * (uint64_t)(S.dims * S.mbits + sumG);
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
  uint32_t Sb = dims * mbits;
  for (uint32_t d = 0; d < dims; ++d) Sb += G[d];
  const uint64_t nwords = (P->meta_bits + 63) / 64;
  const LeafRec* leaves = leaves0 + S.leaf_off;
  uint64_t* meta = (uint64_t*)(S.out + kHeaderBytes);
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
__device__ inline u128 member_code(const KT* keys, uint64_t n, uint32_t dims, const LeafRec& rec,
                                   uint64_t slot) {
  u128 v = 0;
  uint32_t at = 0;
  for (uint32_t d = 0; d < dims; ++d) {
    const uint32_t m = (rec.m >> (8 * d)) & 0xffu;
    if (m == 0) continue;
    const uint32_t q = keys[(uint64_t)d * n + slot];
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

template <typename KT>
__device__ void pack_payload_body(const SetDesc& S, const DevParams* P, uint64_t lb, uint64_t nblk,
                                  const LeafRec* leaves, const uint64_t* off, const KT* keys,
                                  uint64_t* s_off) {
  __shared__ uint64_t s_lo, s_cnt;
  const uint64_t n = S.n, nl = S.n_leaves, base = P->payload_base;
  const uint32_t dims = S.dims;
  const uint64_t nwords = (P->payload_bits + 63) / 64;
  uint64_t* pay = (uint64_t*)(S.out + kHeaderBytes + ((P->meta_bits + 63) / 64) * 8);
  const uint64_t ngroups = (nwords + kBlock - 1) / kBlock;
  for (uint64_t grp = lb; grp < ngroups; grp += nblk) {
    const uint64_t W0 = grp * kBlock;
    const uint64_t Wend = W0 + kBlock < nwords ? W0 + kBlock : nwords;
    if (threadIdx.x == 0) {
      const uint64_t lo = search_off(off, base, 0, nl - 1, W0 * 64);
      const uint64_t hi = search_off(off, base, lo, nl - 1, Wend * 64 - 1);
      s_lo = lo;
      s_cnt = hi - lo + 1;
    }
    __syncthreads();
    const uint64_t lo = s_lo, cnt = s_cnt;
    const bool in_lds = cnt <= 2048;
    if (in_lds)
      for (uint64_t t = threadIdx.x; t < cnt; t += kBlock) s_off[t] = off[lo + t] - base;
    __syncthreads();
    const uint64_t w = W0 + threadIdx.x;
    if (w < Wend) {
      const uint64_t b0 = w * 64;
      uint64_t i;
      if (in_lds) {
        uint64_t a = 0, z = cnt - 1;
        while (a < z) {
          const uint64_t mid = a + (z - a + 1) / 2;
          if (s_off[mid] <= b0)
            a = mid;
          else
            z = mid - 1;
        }
        i = lo + a;
      } else {
        i = search_off(off, base, lo, lo + cnt - 1, b0);
      }
      LeafRec rec = leaves[i];
      uint32_t sm = sum_m(rec.m);
      const uint64_t oi = off[i] - base;
      uint64_t jm = sm ? (b0 - oi) / sm : 0;
      uint64_t at = oi + jm * sm;
      uint64_t word = 0;
      while (at < b0 + 64) {
        if (sm > 0 && jm + 1 < rec.size) {
          const u128 c = member_code(keys, n, dims, rec, (uint64_t)rec.start + 1 + jm);
          or_into(word, b0, c, at, sm);
          at += sm;
          ++jm;
        } else {
          ++i;
          if (i >= nl) break;
          rec = leaves[i];
          sm = sum_m(rec.m);
          jm = 0;
        }
      }
      pay[w] = word;
    }
    __syncthreads();
  }
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
  __shared__ uint64_t s_off[2048];
  const uint64_t lb = blockIdx.x - pre[s], nblk = pre[s + 1] - pre[s];
  const uint8_t* keys = (S.final_buf ? keys1 : keys0) + S.key_off;
  const LeafRec* leaves = leaves0 + S.leaf_off;
  const uint64_t* off = off0 + S.leaf_off;
  if (P->key16)
    pack_payload_body<uint16_t>(S, P, lb, nblk, leaves, off, (const uint16_t*)keys, s_off);
  else
    pack_payload_body<uint32_t>(S, P, lb, nblk, leaves, off, (const uint32_t*)keys, s_off);
}

__global__ void k_header(const SetDesc* sets, const DevParams* params) {
  const SetDesc& S = sets[blockIdx.x];
  const DevParams* P = params + blockIdx.x;
  if (P->status != BBX_OK) return;
  if (threadIdx.x != 0) return;
  const uint32_t dims = S.dims;
  uint64_t h[16];
  for (int k = 0; k < 16; ++k) h[k] = 0;
  h[0] = (uint64_t)kMagic | ((uint64_t)1 << 32) | ((uint64_t)S.dtype << 48) | ((uint64_t)dims << 56);
  h[1] = S.n;
  h[2] = (uint64_t)S.r | ((uint64_t)S.eb_mode << 32) | ((uint64_t)S.mbits << 56);
  h[3] = __double_as_longlong(P->eb_user);
  h[4] = __double_as_longlong(P->eb_abs);
  h[5] = __double_as_longlong(P->eb_eff);
  h[6] = __double_as_longlong(P->w);
  h[7] = __double_as_longlong(P->inv_w);
  for (uint32_t d = 0; d < 3; ++d) h[8 + d] = d < dims ? __double_as_longlong(P->lo[d]) : 0;
  h[11] = (uint64_t)P->G[0] | ((uint64_t)(dims > 1 ? P->G[1] : 0) << 8) |
          ((uint64_t)(dims > 2 ? P->G[2] : 0) << 16);
  h[12] = S.n_leaves;
  h[13] = P->meta_bits;
  h[14] = P->payload_bits;
  h[15] = 0;
  uint64_t* o = (uint64_t*)S.out;
  for (int k = 0; k < 16; ++k) o[k] = h[k];
}

__global__ void k_finish(uint32_t nsets, const SetDesc* sets, const DevParams* params) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsets) return;
  const SetDesc& S = sets[s];
  const uint32_t st = params[s].status;
  if (S.d_size) *S.d_size = st == BBX_OK ? params[s].total_bytes : ~0ull;
  if (S.d_status) *S.d_status = st;
}

hipError_t launch_pack(const BatchPlan& bp, const Ws& w, hipStream_t s) {
  hipError_t e = scan_launch(bp.total_leaves, w.leaf_bits, w.scan_part, w.scan_total, nullptr, 0, s);
  if (e != hipSuccess) return e;
  const uint32_t g = (bp.nsets + kBlock - 1) / kBlock;
  BBX_LAUNCH("set_sizes", k_set_sizes, g, kBlock, 0, s, bp.nsets, w.sets, w.params, w.leaf_bits,
             bp.total_leaves, w.scan_total);
  if (bp.g_pm > 0)
    BBX_LAUNCH("pack_meta", k_pack_meta, bp.g_pm, kBlock, 0, s, bp.nsets, w.pre + bp.o_pm, w.sets,
               w.params, w.leaves);
  if (bp.g_pp > 0)
    BBX_LAUNCH("pack_payload", k_pack_payload, bp.g_pp, kBlock, 0, s, bp.nsets, w.pre + bp.o_pp,
               w.sets, w.params, w.leaves, w.leaf_bits, w.keys[0], w.keys[1]);
  BBX_LAUNCH("header", k_header, bp.nsets, 64, 0, s, w.sets, w.params);
  BBX_LAUNCH("finish", k_finish, g, kBlock, 0, s, bp.nsets, w.sets, w.params);
  return hipGetLastError();
}

}  // namespace bbx

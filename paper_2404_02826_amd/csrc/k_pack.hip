// k_pack.hip -- leaf bit offsets and bit packing (Sec. 4.2, storage layout).
//
//   k_scan_reduce / k_scan_top / k_scan_down
//        exclusive prefix sum of the per-leaf payload bits (depth-first
//        order), in place; the top pass also fixes the section sizes:
//        meta = n_leaves * (dims*mbits + sum G_d) bits, payload = the total
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

__global__ void __launch_bounds__(kBlock) k_scan_reduce(uint64_t count, const uint64_t* bits,
                                                        uint64_t* part, const DevParams* P) {
  if (P->status != BBX_OK) return;
  const uint64_t base = blockIdx.x * kScanChunk + (uint64_t)threadIdx.x * kScanPer;
  uint64_t s = 0;
  for (int k = 0; k < kScanPer; ++k)
    if (base + k < count) s += bits[base + k];
  uint64_t tot;
  (void)bexscan(s, &tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// mode 0 (compress): record the section sizes, check out_cap.
// mode 1 (decompress): the total must equal the header's payload bits.
__global__ void __launch_bounds__(kBlock) k_scan_top(uint64_t nparts, uint64_t* part,
                                                     DevParams* P, uint32_t mode,
                                                     uint64_t n_leaves, uint32_t dims,
                                                     uint32_t mbits, uint64_t out_cap,
                                                     uint64_t expect_payload) {
  if (P->status != BBX_OK) return;
  const uint64_t per = (nparts + kBlock - 1) / kBlock;
  const uint64_t b0 = threadIdx.x * per;
  uint64_t s = 0;
  for (uint64_t k = 0; k < per; ++k)
    if (b0 + k < nparts) s += part[b0 + k];
  uint64_t tot;
  uint64_t run = bexscan(s, &tot);
  for (uint64_t k = 0; k < per; ++k)
    if (b0 + k < nparts) {
      uint64_t v = part[b0 + k];
      part[b0 + k] = run;
      run += v;
    }
  if (threadIdx.x == 0) {
    if (mode == 0) {
      uint32_t sumG = 0;
      for (uint32_t d = 0; d < dims; ++d) sumG += P->G[d];
      const uint64_t meta = n_leaves * (uint64_t)(dims * mbits + sumG);
      P->meta_bits = meta;
      P->payload_bits = tot;
      P->total_bytes = kHeaderBytes + ((meta + 63) / 64) * 8 + ((tot + 63) / 64) * 8;
      if (P->total_bytes > out_cap) P->status = BBX_ENOSPC;
    } else {
      if (tot != expect_payload) P->status = BBX_ECORRUPT;
      P->payload_bits = tot;
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_scan_down(uint64_t count, uint64_t* bits,
                                                      const uint64_t* part, const DevParams* P) {
  if (P->status != BBX_OK) return;
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

hipError_t launch_scan(uint64_t count, uint64_t* bits, uint64_t* part, DevParams* params,
                       const CompressPlan* cp, uint64_t expect_payload, size_t out_cap,
                       uint64_t* /*d_size*/, hipStream_t s) {
  const uint64_t nb = scan_blocks(count);
  if (nb > 0)
    BBX_LAUNCH("scan_reduce", k_scan_reduce, nb, kBlock, 0, s, count, bits, part, params);
  BBX_LAUNCH("scan_top", k_scan_top, 1, kBlock, 0, s, nb, part, params, cp ? 0u : 1u, count,
             cp ? cp->dims : 0u, cp ? cp->mbits : 0u, (uint64_t)out_cap, expect_payload);
  if (nb > 0) BBX_LAUNCH("scan_down", k_scan_down, nb, kBlock, 0, s, count, bits, part, params);
  return hipGetLastError();
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

__global__ void __launch_bounds__(kBlock) k_pack_meta(uint64_t n_leaves, uint32_t dims,
                                                      uint32_t mbits, const DevParams* P,
                                                      const LeafRec* leaves, uint8_t* out) {
  if (P->status != BBX_OK) return;
  uint32_t G[3] = {P->G[0], P->G[1], P->G[2]};
  uint32_t S = dims * mbits;
  for (uint32_t d = 0; d < dims; ++d) S += G[d];
  const uint64_t nwords = (P->meta_bits + 63) / 64;
  uint64_t* meta = (uint64_t*)(out + kHeaderBytes);
  for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < nwords;
       w += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t b0 = w * 64;
    uint64_t i0 = b0 / S, i1 = (b0 + 63) / S;
    if (i1 >= n_leaves) i1 = n_leaves - 1;
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
      or_into(word, b0, v, i * S, S);
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

// largest i in [lo, hi] with off[i] <= b (off non-decreasing, off[lo] <= b)
__device__ inline uint64_t search_off(const uint64_t* off, uint64_t lo, uint64_t hi, uint64_t b) {
  while (lo < hi) {
    uint64_t mid = lo + (hi - lo + 1) / 2;
    if (off[mid] <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

template <typename KT>
__device__ void pack_payload_body(uint64_t n, uint32_t dims, uint64_t n_leaves,
                                  const DevParams* P, const LeafRec* leaves, const uint64_t* off,
                                  const KT* keys, uint8_t* out, uint64_t* s_off) {
  __shared__ uint64_t s_lo, s_cnt;
  const uint64_t total = P->payload_bits;
  const uint64_t nwords = (total + 63) / 64;
  uint64_t* pay = (uint64_t*)(out + kHeaderBytes + ((P->meta_bits + 63) / 64) * 8);
  const uint64_t ngroups = (nwords + kBlock - 1) / kBlock;
  for (uint64_t grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
    const uint64_t W0 = grp * kBlock;
    const uint64_t Wend = W0 + kBlock < nwords ? W0 + kBlock : nwords;
    if (threadIdx.x == 0) {
      uint64_t lo = search_off(off, 0, n_leaves - 1, W0 * 64);
      uint64_t hi = search_off(off, lo, n_leaves - 1, Wend * 64 - 1);
      s_lo = lo;
      s_cnt = hi - lo + 1;
    }
    __syncthreads();
    const uint64_t lo = s_lo, cnt = s_cnt;
    const bool in_lds = cnt <= 2048;
    if (in_lds)
      for (uint64_t t = threadIdx.x; t < cnt; t += kBlock) s_off[t] = off[lo + t];
    __syncthreads();
    const uint64_t w = W0 + threadIdx.x;
    if (w < Wend) {
      const uint64_t b0 = w * 64;
      uint64_t i;
      if (in_lds) {
        uint64_t a = 0, z = cnt - 1;
        while (a < z) {
          uint64_t mid = a + (z - a + 1) / 2;
          if (s_off[mid] <= b0)
            a = mid;
          else
            z = mid - 1;
        }
        i = lo + a;
      } else {
        i = search_off(off, lo, lo + cnt - 1, b0);
      }
      LeafRec rec = leaves[i];
      uint32_t sm = sum_m(rec.m);
      uint64_t oi = off[i];
      uint64_t jm = sm ? (b0 - oi) / sm : 0;
      uint64_t at = oi + jm * sm;
      uint64_t word = 0;
      while (at < b0 + 64) {
        if (sm > 0 && jm + 1 < rec.size) {
          u128 c = member_code(keys, n, dims, rec, (uint64_t)rec.start + 1 + jm);
          or_into(word, b0, c, at, sm);
          at += sm;
          ++jm;
        } else {
          ++i;
          if (i >= n_leaves) break;
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

__global__ void __launch_bounds__(kBlock) k_pack_payload(uint64_t n, uint32_t dims,
                                                         uint64_t n_leaves, const DevParams* P,
                                                         const LeafRec* leaves,
                                                         const uint64_t* off, const void* keys,
                                                         uint8_t* out) {
  if (P->status != BBX_OK) return;
  if (P->payload_bits == 0) return;
  __shared__ uint64_t s_off[2048];
  if (P->key16)
    pack_payload_body<uint16_t>(n, dims, n_leaves, P, leaves, off, (const uint16_t*)keys, out,
                                s_off);
  else
    pack_payload_body<uint32_t>(n, dims, n_leaves, P, leaves, off, (const uint32_t*)keys, out,
                                s_off);
}

__global__ void k_header(uint64_t n, uint32_t dims, uint32_t dtype, uint32_t r, uint32_t eb_mode,
                         uint32_t mbits, uint64_t n_leaves, const DevParams* P, uint8_t* out) {
  if (P->status != BBX_OK) return;
  if (threadIdx.x != 0) return;
  uint64_t h[16];
  for (int k = 0; k < 16; ++k) h[k] = 0;
  h[0] = (uint64_t)kMagic | ((uint64_t)1 << 32) | ((uint64_t)dtype << 48) | ((uint64_t)dims << 56);
  h[1] = n;
  h[2] = (uint64_t)r | ((uint64_t)eb_mode << 32) | ((uint64_t)mbits << 56);
  h[3] = __double_as_longlong(P->eb_user);
  h[4] = __double_as_longlong(P->eb_abs);
  h[5] = __double_as_longlong(P->eb_eff);
  h[6] = __double_as_longlong(P->w);
  h[7] = __double_as_longlong(P->inv_w);
  for (uint32_t d = 0; d < 3; ++d) h[8 + d] = d < dims ? __double_as_longlong(P->lo[d]) : 0;
  h[11] = (uint64_t)(dims > 0 ? P->G[0] : 0) | ((uint64_t)(dims > 1 ? P->G[1] : 0) << 8) |
          ((uint64_t)(dims > 2 ? P->G[2] : 0) << 16);
  h[12] = n_leaves;
  h[13] = P->meta_bits;
  h[14] = P->payload_bits;
  h[15] = 0;
  uint64_t* o = (uint64_t*)out;
  for (int k = 0; k < 16; ++k) o[k] = h[k];
}

__global__ void k_finish(const DevParams* P, uint64_t* d_size, uint32_t* d_status) {
  if (threadIdx.x != 0) return;
  const uint32_t st = P->status;
  if (d_size) *d_size = st == BBX_OK ? P->total_bytes : ~0ull;
  if (d_status) *d_status = st;
}

hipError_t launch_pack(const CompressPlan& p, const CompressWs& w, int buf, uint8_t* out,
                       uint64_t* d_size, uint32_t* d_status, hipStream_t s) {
  if (p.n_leaves > 0) {
    uint64_t meta_words_max = (p.n_leaves * (uint64_t)(p.dims * (p.mbits + 30)) + 63) / 64;
    uint64_t g = (meta_words_max + kBlock - 1) / kBlock;
    if (g > 2048) g = 2048;
    if (g == 0) g = 1;
    BBX_LAUNCH("pack_meta", k_pack_meta, g, kBlock, 0, s, p.n_leaves, p.dims, p.mbits, w.params,
               w.leaves, out);
    uint64_t pay_words_max = (p.n * (uint64_t)p.dims * 31 + 63) / 64;
    uint64_t g2 = (pay_words_max + kBlock - 1) / kBlock;
    if (g2 > 4096) g2 = 4096;
    if (g2 == 0) g2 = 1;
    BBX_LAUNCH("pack_payload", k_pack_payload, g2, kBlock, 0, s, p.n, p.dims, p.n_leaves,
               w.params, w.leaves, w.leaf_bits, w.keys[buf], out);
  }
  BBX_LAUNCH("header", k_header, 1, 64, 0, s, p.n, p.dims, p.dtype, p.r, p.eb_mode, p.mbits,
             p.n_leaves, w.params, out);
  BBX_LAUNCH("finish", k_finish, 1, 64, 0, s, w.params, d_size, d_status);
  return hipGetLastError();
}

}  // namespace bbx

// k_unpack.hip -- unpack and dequantize (Sec. 3: reconstruction at the bin
// centre origin + q*w, FP64 multiply then add, then rounding to the type).
//
//   k_dec_meta   one thread per leaf: reads its fixed-stride meta record,
//                validates the widths, and derives its span from (n, r) alone
//                (the tree's leaf sizes depend on n and r only); with
//                ref_mode 1 the reference's code comes from its stored
//                coordinates by the quantization of Sec. 3
//   (scan)       payload bit offset of every leaf, total checked against the
//                header
//   k_unpack     blocks of 1024 output slots: the block finds the leaves that
//                cover its slots, every thread decodes slots
//                (reference -> its code; member j -> payload code j-1)
//   k_dec_refs   ref_mode 1: the references' stored coordinates, exactly
//   k_export     the Sec. 4.2 sequence layout of a ref_mode 1 stream (with
//                k_dec_meta and the scan for the leaves' code offsets)
#include "bbx_internal.h"

namespace bbx {

typedef unsigned __int128 u128;

__device__ inline u128 read_bits(const uint64_t* sec, uint64_t nwords, uint64_t at, uint32_t len) {
  if (len == 0) return 0;
  const uint64_t w0 = at >> 6;
  const uint32_t s = (uint32_t)(at & 63);
  u128 v = (u128)sec[w0];
  if (w0 + 1 < nwords) v |= (u128)sec[w0 + 1] << 64;
  v >>= s;
  if (s + len > 128 && w0 + 2 < nwords) v |= (u128)sec[w0 + 2] << (128 - s);
  if (len < 128) v &= (((u128)1) << len) - 1;
  return v;
}

// Reference field of a ref_mode 1 record: the stored coordinate of axis d
// (M bits at absolute bit `at`), and the code the encoder's quantization gave
// it: floor((x - origin) * inv_w + 1/2) in FP64, the same separately rounded
// operations as the quantize pass (no contraction).  Returns false when the
// value is not finite or its code lies outside [0, 2^G).
__device__ inline bool ref_code_from_coord(const uint64_t* meta, uint64_t nwords, uint64_t at,
                                           uint32_t dtype, double origin, double inv_w,
                                           uint32_t G, uint32_t* q) {
  const uint64_t raw = (uint64_t)read_bits(meta, nwords, at, coord_bits(dtype));
  const double x = dtype == BBX_F32 ? (double)__uint_as_float((uint32_t)raw) : __longlong_as_double((long long)raw);
  if (!isfinite(x)) return false;
  const double t = floor((x - origin) * inv_w + 0.5);
  if (!(t >= 0.0 && t < (double)(1ull << G))) return false;
  *q = (uint32_t)t;
  return true;
}

__global__ void __launch_bounds__(kBlock) k_dec_meta(uint64_t n_leaves, uint32_t dims,
                                                     uint32_t mbits, uint32_t G0, uint32_t G1,
                                                     uint32_t G2, uint64_t meta_bits, TreeGeom g,
                                                     const uint8_t* stream, LeafRec* leaves,
                                                     uint64_t* bits, DevParams* P,
                                                     uint32_t ref_mode, uint32_t dtype, double o0,
                                                     double o1, double o2, double inv_w) {
  const uint32_t G[3] = {G0, G1, G2};
  const double origin[3] = {o0, o1, o2};
  uint32_t S = dims * mbits;
  for (uint32_t d = 0; d < dims; ++d) S += ref_mode ? coord_bits(dtype) : G[d];
  const uint64_t* meta = (const uint64_t*)(stream + kHeaderBytes);
  const uint64_t nwords = (meta_bits + 63) / 64;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_leaves;
       i += (uint64_t)gridDim.x * blockDim.x) {
    // widths (and with ref_mode 0 the reference codes) in one read: at most
    // 3 * (6 + 30) bits
    u128 v = read_bits(meta, nwords, i * S, ref_mode ? dims * mbits : S);
    LeafRec rec;
    uint32_t m = 0, summ = 0;
    bool bad = false;
    for (uint32_t d = 0; d < dims; ++d) {
      uint32_t md = (uint32_t)(v & ((1u << mbits) - 1));
      v >>= mbits;
      if (md == 1 || md > 31 || md > G[d] + 1) bad = true;
      m |= md << (8 * d);
      summ += md;
    }
    for (uint32_t d = 0; d < 3; ++d) {
      rec.qref[d] = 0;
      if (d < dims && ref_mode) {
        const uint64_t at = i * S + dims * mbits + d * coord_bits(dtype);
        if (!ref_code_from_coord(meta, nwords, at, dtype, origin[d], inv_w, G[d], &rec.qref[d]))
          bad = true;
      } else if (d < dims) {
        rec.qref[d] = (uint32_t)(v & ((((u128)1) << G[d]) - 1));
        v >>= G[d];
      }
    }
    rec.ref_src = 0;
    uint64_t st, sz;
    leaf_span(g, i, &st, &sz);
    rec.start = (uint32_t)st;
    rec.size = (uint32_t)sz;
    rec.m = m;
    leaves[i] = rec;
    bits[i] = bad ? 0 : (sz - 1) * (uint64_t)summ;
    if (bad) P->status = BBX_ECORRUPT;
  }
}

constexpr uint32_t kLeafStage = 256;     // leaves per block (leaves_per_block)
constexpr uint32_t kUnpackWords = 1534;  // staged payload words per block (+2 zero words: 12 KB)
constexpr uint32_t kMapGroups = 520;     // 4-slot groups of a block's leaf map (2,048 slots and the ends)

// Leaf-aligned decoding: a block takes leaves_per_block(r) consecutive
// leaves, stages their records, bit offsets and payload words with coalesced
// loads, and decodes their slots (reference -> its code; member j -> payload
// code j-1) from LDS.
// up to 64 bits at absolute bit `at` of a word array (the words exist)
__device__ inline uint64_t read64(const uint64_t* sec, uint64_t at, uint32_t len) {
  const uint64_t w = at >> 6;
  const uint32_t s = (uint32_t)(at & 63);
  uint64_t v = sec[w] >> s;
  if (s + len > 64) v |= sec[w + 1] << (64 - s);
  return len < 64 ? v & ((1ull << len) - 1) : v;
}

template <typename T, int DIMS>
__device__ void unpack_body(uint64_t n, uint32_t layout, uint32_t r, double w,
                            const double* origin, const uint32_t* G, uint64_t nl,
                            const LeafRec* leaves, const uint64_t* off, const uint64_t* pay,
                            uint64_t pay_words, uint64_t pbits, T* out, DevParams* P,
                            LeafRec* s_rec, uint64_t* s_off, uint64_t* s_pay, uint16_t* s_map) {
  constexpr uint32_t dims = DIMS;
  const uint32_t lpb = leaves_per_block(r);
  const uint64_t L0 = (uint64_t)blockIdx.x * lpb;
  if (L0 >= nl) return;
  const uint32_t nlb = (uint32_t)(nl - L0 < lpb ? nl - L0 : lpb);
  for (uint32_t t = threadIdx.x; t < nlb; t += kBlock) {
    s_rec[t] = leaves[L0 + t];
    s_off[t] = off[L0 + t];
  }
  const uint64_t bo1 = L0 + nlb < nl ? off[L0 + nlb] : pbits;
  __syncthreads();
  // leaf map: the leaf holding the first slot of each 4-aligned group of
  // slots (each leaf writes the groups that start inside it), when the
  // block's slots fit the map
  const uint64_t mbase = (uint64_t)s_rec[0].start & ~3ull;
  const uint64_t mend = (uint64_t)s_rec[nlb - 1].start + s_rec[nlb - 1].size;
  const bool mapped = mend - mbase <= 4ull * kMapGroups;
  if (mapped)
    for (uint32_t t = threadIdx.x; t < nlb; t += kBlock) {
      const uint64_t st = s_rec[t].start - mbase, en = st + s_rec[t].size;
      for (uint64_t g = (st + 3) >> 2; 4 * g < en; ++g) s_map[g] = (uint16_t)t;
    }
  const uint64_t bo0 = s_off[0];
  const uint64_t w0 = bo0 / 64, w1 = bo1 > bo0 ? (bo1 + 63) / 64 : w0;
  const bool staged = w1 - w0 <= kUnpackWords;
  const uint32_t nw = staged ? (uint32_t)(w1 - w0) : 0u;
  for (uint32_t t = threadIdx.x; t < nw; t += kBlock) s_pay[t] = w0 + t < pay_words ? pay[w0 + t] : 0;
  if (threadIdx.x < 2) s_pay[nw + threadIdx.x] = 0;  // read past the end, then unused
  __syncthreads();
  const uint64_t slot0 = s_rec[0].start;
  const uint64_t slot1 = (uint64_t)s_rec[nlb - 1].start + s_rec[nlb - 1].size;
  bool corrupt = false;
  // each thread decodes 4 consecutive slots (4-aligned slot indices); with an
  // aligned array-of-structures output the 4 particles go out as whole
  // 16-byte stores
  const bool vec = layout == BBX_AOS && ((uintptr_t)out & 15) == 0;
  // staged payload, 16-byte AoS stores, and every member within 64 code bits
  // (m_d <= G_d + 1, so sum_d (G_d + 1) <= 64 bounds every leaf): the four
  // slots of a thread decode without branches (below)
  uint32_t gsum = 0;
#pragma unroll
  for (uint32_t d = 0; d < DIMS; ++d) gsum += G[d] + 1;
  const bool simple = staged && vec && gsum <= 64;
  const uint32_t bit0 = (uint32_t)(w0 * 64);  // staged bit offsets fit 32 bits
  for (uint64_t gs = (slot0 & ~3ull) + 4ull * threadIdx.x; gs < slot1; gs += 4ull * kBlock) {
    const bool full = vec && gs >= slot0 && gs + 4 <= slot1;
    union {
      T e[4 * DIMS];
      uint4 v[4 * DIMS * sizeof(T) / 16];
    } o;
    if (simple && full) {
      uint32_t a = 0, z = nlb - 1;  // last staged leaf starting at or before gs
      if (mapped) {
        a = s_map[(gs - mbase) >> 2];
      } else {
        while (a < z) {
          const uint32_t mid = (a + z + 1) >> 1;
          if (s_rec[mid].start <= gs)
            a = mid;
          else
            z = mid - 1;
        }
      }
#pragma unroll
      for (uint32_t k = 0; k < 4; ++k) {
        const uint32_t p = (uint32_t)(gs + k);
        while (a + 1 < nlb && s_rec[a + 1].start <= p) ++a;
        const LeafRec rec = s_rec[a];
        const uint32_t j = p - rec.start;
        const uint32_t mm[3] = {rec.m & 0xffu, DIMS > 1 ? (rec.m >> 8) & 0xffu : 0u,
                                DIMS > 2 ? (rec.m >> 16) & 0xffu : 0u};
        const uint32_t summ = mm[0] + mm[1] + mm[2];
        // member j > 0 holds payload code j - 1; the reference reads a code
        // it does not use
        const uint32_t at = (uint32_t)s_off[a] - bit0 + (j ? j - 1 : 0u) * summ;
        const uint32_t wi = at >> 6, sh = at & 63u;
        const uint64_t lo = s_pay[wi], hi = s_pay[wi + 1];
        const uint64_t v = sh ? (lo >> sh) | (hi << (64 - sh)) : lo;
        const uint32_t fo[3] = {0u, mm[0], mm[0] + mm[1]};
#pragma unroll
        for (uint32_t d = 0; d < DIMS; ++d) {
          const uint32_t half = (1u << mm[d]) >> 1;
          const uint32_t u = (uint32_t)(v >> fo[d]) & ((1u << mm[d]) - 1u);
          if (j && mm[d] && !u) corrupt = true;
          const int64_t q = (int64_t)rec.qref[d] + (j ? (int64_t)u - (int64_t)half : 0);
          uint32_t qq = (uint32_t)q;
          if ((uint64_t)q >= (1ull << G[d])) {
            corrupt = true;
            qq = 0;
          }
          o.e[k * DIMS + d] = (T)(origin[d] + (double)qq * w);
        }
      }
      uint4* dst = (uint4*)(out + gs * dims);
#pragma unroll
      for (uint32_t i = 0; i < 4 * DIMS * sizeof(T) / 16; ++i) dst[i] = o.v[i];
      continue;
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
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) {
      const uint64_t p = gs + k;
      if (p < slot0 || p >= slot1) continue;
      while (a + 1 < nlb && s_rec[a + 1].start <= p) ++a;
      const LeafRec rec = s_rec[a];
      const uint32_t j = (uint32_t)(p - rec.start);
      // widths (m_d <= 31: the meta check rejects wider); m_d = 0 gives a
      // zero mask and a zero offset, so such an axis keeps the reference code
      const uint32_t m0 = rec.m & 0xffu, m1 = dims > 1 ? (rec.m >> 8) & 0xffu : 0u,
                     m2 = dims > 2 ? (rec.m >> 16) & 0xffu : 0u;
      const uint32_t summ = m0 + m1 + m2;
      uint32_t u[3] = {0, 0, 0};
      const uint32_t mm[3] = {m0, m1, m2};
      if (j > 0) {
        const uint64_t at = s_off[a] + (uint64_t)(j - 1) * summ;
        if (summ <= 64) {
          const uint64_t v = staged ? read64(s_pay, at - w0 * 64, summ) : read64(pay, at, summ);
          u[0] = (uint32_t)v & ((1u << m0) - 1);
          u[1] = (uint32_t)(v >> m0) & ((1u << m1) - 1);
          u[2] = (uint32_t)(v >> (m0 + m1)) & ((1u << m2) - 1);
        } else {
          u128 v = staged ? read_bits(s_pay, nw, at - w0 * 64, summ) : read_bits(pay, pay_words, at, summ);
#pragma unroll
          for (uint32_t d = 0; d < 3; ++d) {
            u[d] = (uint32_t)(v & ((((u128)1) << mm[d]) - 1));
            v >>= mm[d];
          }
        }
#pragma unroll
        for (uint32_t d = 0; d < 3; ++d)
          if (d < dims && mm[d] != 0 && u[d] == 0) corrupt = true;
      }
#pragma unroll
      for (uint32_t d = 0; d < 3; ++d) {
        if (d >= dims) break;
        // q = q_ref + u - 2^(m-1) for a member, q_ref for the reference
        const int64_t q = (int64_t)rec.qref[d] + (j > 0 ? (int64_t)u[d] - (int64_t)((1u << mm[d]) >> 1) : 0);
        uint32_t qq = (uint32_t)q;
        if ((uint64_t)q >= (1ull << G[d])) {
          corrupt = true;
          qq = 0;
        }
        const double x = origin[d] + (double)qq * w;
        const T t = (T)x;
        if (full)
          o.e[k * dims + d] = t;
        else if (layout == BBX_AOS)
          out[p * dims + d] = t;
        else
          out[(uint64_t)d * n + p] = t;
      }
    }
    if (full) {
      uint4* dst = (uint4*)(out + gs * dims);
#pragma unroll
      for (uint32_t i = 0; i < 4 * DIMS * sizeof(T) / 16; ++i) dst[i] = o.v[i];
    }
  }
  if (corrupt) P->status = BBX_ECORRUPT;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_unpack(uint64_t n, uint32_t dims, uint32_t layout,
                                                   uint32_t r, double w, double o0, double o1,
                                                   double o2, uint32_t G0, uint32_t G1,
                                                   uint32_t G2, uint64_t n_leaves,
                                                   uint64_t meta_bits, const LeafRec* leaves,
                                                   const uint64_t* off, const uint8_t* stream,
                                                   uint64_t pay_bits, T* out, DevParams* P) {
  if (P->status != BBX_OK) return;
  __shared__ LeafRec s_rec[kLeafStage];
  __shared__ uint64_t s_off[kLeafStage];
  __shared__ uint64_t s_pay[kUnpackWords + 2];
  __shared__ uint16_t s_map[kMapGroups];
  const double origin[3] = {o0, o1, o2};
  const uint32_t G[3] = {G0, G1, G2};
  const uint64_t* pay = (const uint64_t*)(stream + kHeaderBytes + ((meta_bits + 63) / 64) * 8);
  if (dims == 3)
    unpack_body<T, 3>(n, layout, r, w, origin, G, n_leaves, leaves, off, pay, (pay_bits + 63) / 64,
                      pay_bits, out, P, s_rec, s_off, s_pay, s_map);
  else
    unpack_body<T, 2>(n, layout, r, w, origin, G, n_leaves, leaves, off, pay, (pay_bits + 63) / 64,
                      pay_bits, out, P, s_rec, s_off, s_pay, s_map);
}

// Starts a decode: clears the status and checks that the stream's own
// header is the one the launch was planned from (one 8-byte word per lane).
__global__ void k_dec_init(DevParams* P, const uint8_t* stream, HeaderCopy h) {
  const uint32_t lane = threadIdx.x;
  const bool diff = lane < kHeaderBytes / 8 && ((const uint64_t*)stream)[lane] != h.w[lane];
  const uint64_t any = __ballot(diff);
  if (lane == 0) {
    P->status = any ? BBX_ECORRUPT : BBX_OK;
    P->payload_bits = 0;
  }
}

__global__ void k_dec_finish(const DevParams* P, uint32_t* d_status) {
  if (threadIdx.x == 0 && d_status) *d_status = P->status;
}

// ref_mode 1: each leaf's first output slot (its reference, where k_unpack
// wrote the bin centre of its code) receives the stored original
// coordinates, bit for bit.  One thread per leaf.
template <typename U>
__global__ void __launch_bounds__(kBlock) k_dec_refs(uint64_t n, uint64_t n_leaves, uint32_t dims,
                                                     uint32_t mbits, uint32_t layout,
                                                     uint64_t meta_bits, const LeafRec* leaves,
                                                     const uint8_t* stream, U* pos,
                                                     const DevParams* P) {
  if (P->status != BBX_OK) return;
  constexpr uint32_t M = 8 * sizeof(U);
  const uint32_t S = dims * (mbits + M);
  const uint64_t* meta = (const uint64_t*)(stream + kHeaderBytes);
  const uint64_t nwords = (meta_bits + 63) / 64;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_leaves;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t st = leaves[i].start;
    for (uint32_t d = 0; d < dims; ++d) {
      const U raw = (U)read_bits(meta, nwords, i * S + dims * mbits + d * M, M);
      pos[layout == BBX_AOS ? st * dims + d : (uint64_t)d * n + st] = raw;
    }
  }
}

// A lossless stream: the stored bits of every coordinate, in input order.
__global__ void __launch_bounds__(kBlock) k_unpack_lossless(uint64_t n, uint32_t dims, uint32_t dtype,
                                                            uint32_t layout, const uint8_t* stream,
                                                            void* pos, const DevParams* P) {
  if (P->status != BBX_OK) return;
  const uint64_t nv = n * dims;
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nv;
       k += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t i = k / dims, d = k - i * dims;
    const uint64_t o = layout == BBX_AOS ? k : d * n + i;
    if (dtype == BBX_F32)
      ((uint32_t*)pos)[o] = ((const uint32_t*)(stream + kHeaderBytes))[k];
    else
      ((uint64_t*)pos)[o] = ((const uint64_t*)(stream + kHeaderBytes))[k];
  }
}

hipError_t launch_decompress(const DecompressPlan& p, const DecompressWs& w, const uint8_t* stream,
                             void* pos, uint32_t* d_status, hipStream_t s) {
  BBX_LAUNCH("dec_init", k_dec_init, 1, 64, 0, s, w.params, stream, p.header);
  if (p.n > 0 && p.version == 3) {
    uint64_t g = (p.n * p.dims + kBlock - 1) / kBlock;
    if (g > 16384) g = 16384;
    BBX_LAUNCH("unpack_lossless", k_unpack_lossless, g, kBlock, 0, s, p.n, p.dims, p.dtype,
               p.layout, stream, pos, w.params);
  } else if (p.n > 0 && p.version == 2) {
    hipError_t e = launch_decompress2(p, w, stream, pos, s);
    if (e != hipSuccess) return e;
  } else if (p.n > 0) {
    uint64_t g = (p.n_leaves + kBlock - 1) / kBlock;
    if (g > 65536) g = 65536;
    BBX_LAUNCH("dec_meta", k_dec_meta, g, kBlock, 0, s, p.n_leaves, p.dims, p.mbits, p.G[0],
               p.G[1], p.G[2], p.meta_bits, p.geom, stream, w.leaves, w.leaf_bits, w.params,
               p.ref_mode, p.dtype, p.origin[0], p.origin[1], p.origin[2], p.inv_w);
    hipError_t e = launch_dec_scan(p.n_leaves, w.leaf_bits, w.scan_part, w.params, p.payload_bits, s);
    if (e != hipSuccess) return e;
    const uint64_t lpb = leaves_per_block(p.r);
    const uint64_t blocks = (p.n_leaves + lpb - 1) / lpb;
    if (p.dtype == BBX_F32)
      BBX_LAUNCH("unpack", k_unpack<float>, blocks, kBlock, 0, s, p.n, p.dims, p.layout, p.r,
                 p.w, p.origin[0], p.origin[1], p.origin[2], p.G[0], p.G[1], p.G[2], p.n_leaves,
                 p.meta_bits, w.leaves, w.leaf_bits, stream, p.payload_bits, (float*)pos,
                 w.params);
    else
      BBX_LAUNCH("unpack", k_unpack<double>, blocks, kBlock, 0, s, p.n, p.dims, p.layout, p.r,
                 p.w, p.origin[0], p.origin[1], p.origin[2], p.G[0], p.G[1], p.G[2], p.n_leaves,
                 p.meta_bits, w.leaves, w.leaf_bits, stream, p.payload_bits, (double*)pos,
                 w.params);
    if (p.ref_mode && p.dtype == BBX_F32)
      BBX_LAUNCH("dec_refs", k_dec_refs<uint32_t>, g, kBlock, 0, s, p.n, p.n_leaves, p.dims,
                 p.mbits, p.layout, p.meta_bits, w.leaves, stream, (uint32_t*)pos, w.params);
    else if (p.ref_mode)
      BBX_LAUNCH("dec_refs", k_dec_refs<uint64_t>, g, kBlock, 0, s, p.n, p.n_leaves, p.dims,
                 p.mbits, p.layout, p.meta_bits, w.leaves, stream, (uint64_t*)pos, w.params);
  }
  BBX_LAUNCH("dec_finish", k_dec_finish, 1, 64, 0, s, w.params, d_status);
  return hipGetLastError();
}

// ---------------------------------------------------------------- sequence export

constexpr uint32_t kExportLeaves = 256;  // leaves per block of k_export

// ORs the low `len` (<= 64) bits of v, whose bit 0 sits at absolute bit
// `at`, into the word whose bit 0 sits at absolute bit w0.
__device__ inline void or_bits(uint64_t& word, uint64_t w0, uint64_t v, uint64_t at, uint32_t len) {
  if (len == 0 || at >= w0 + 64 || at + len <= w0) return;
  if (len < 64) v &= (1ull << len) - 1;
  if (at >= w0)
    word |= v << (at - w0);
  else
    word |= v >> (w0 - at);
}

// Zeroes the output words that two blocks of k_export share (the word
// holding the first bit of every block's first sequence but the first).
// After a failed validation (the offsets may then run past the layout)
// nothing is written.
__global__ void k_export_edges(uint64_t n_leaves, uint64_t F, const uint64_t* off, uint64_t* out,
                               uint64_t out_words, const DevParams* P) {
  if (P->status != BBX_OK) return;
  const uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x + 1;
  const uint64_t L0 = b * kExportLeaves;
  if (L0 >= n_leaves) return;
  const uint64_t at = L0 * F + off[L0];
  if ((at & 63) && (at >> 6) < out_words) out[at >> 6] = 0;
}

// The Sec. 4.2 sequence layout of a ref_mode 1 stream: per leaf, in stored
// order, the centre's coordinate bits (M per axis), the widths (mbits each),
// the member codes (the leaf's payload segment, `off` its exclusive bit
// offsets) and a 32-bit end mark of all ones.  A block takes kExportLeaves
// leaves and writes the output words their sequences cover, one thread per
// word; the words it shares with a neighbouring block (zeroed before) take
// an atomic OR, every other word a plain store.
__global__ void __launch_bounds__(kBlock) k_export(uint64_t n_leaves, uint32_t dims, uint32_t mbits,
                                                   uint32_t M, uint64_t meta_bits,
                                                   uint64_t payload_bits, const uint64_t* off,
                                                   const uint8_t* stream, uint64_t* out,
                                                   const DevParams* P) {
  if (P->status != BBX_OK) return;
  __shared__ uint64_t so[kExportLeaves + 1];  // first output bit of each sequence (+ the end)
  const uint64_t F = (uint64_t)dims * (M + mbits) + 32;  // bits of a sequence besides its codes
  const uint64_t L0 = (uint64_t)blockIdx.x * kExportLeaves;
  const uint32_t cnt = (uint32_t)(n_leaves - L0 < kExportLeaves ? n_leaves - L0 : kExportLeaves);
  for (uint32_t t = threadIdx.x; t <= cnt; t += blockDim.x) {
    const uint64_t L = L0 + t;
    so[t] = L * F + (L < n_leaves ? off[L] : payload_bits);
  }
  __syncthreads();
  const uint64_t* meta = (const uint64_t*)(stream + kHeaderBytes);
  const uint64_t mwords = (meta_bits + 63) / 64;
  const uint64_t* pay = meta + mwords;
  const uint64_t pwords = (payload_bits + 63) / 64;
  const uint64_t S = (uint64_t)dims * (mbits + M);
  const uint64_t b_beg = so[0], b_end = so[cnt];  // b_end - b_beg >= F > 0
  const uint64_t w_first = b_beg >> 6, w_last = (b_end - 1) >> 6;
  for (uint64_t w = w_first + threadIdx.x; w <= w_last; w += blockDim.x) {
    const uint64_t b0 = w << 6;
    // the last sequence starting at or before the word (or the block's first)
    const uint64_t x = b0 > b_beg ? b0 : b_beg;
    uint32_t lo = 0, hi = cnt;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (so[mid] <= x)
        lo = mid;
      else
        hi = mid;
    }
    uint64_t word = 0;
    for (uint32_t i = lo; i < cnt && so[i] < b0 + 64; ++i) {
      const uint64_t L = L0 + i, at = so[i], rec = L * S;
      const uint64_t p0 = at + dims * (M + mbits), plen = so[i + 1] - at - F;
      if (at < b0 + 64 && p0 > b0) {  // centre and widths reach into the word
        for (uint32_t d = 0; d < dims; ++d) {
          or_bits(word, b0, (uint64_t)read_bits(meta, mwords, rec + dims * mbits + d * M, M),
                  at + d * M, M);
          or_bits(word, b0, (uint64_t)read_bits(meta, mwords, rec + d * mbits, mbits),
                  at + dims * M + d * mbits, mbits);
        }
      }
      if (plen && p0 < b0 + 64 && p0 + plen > b0) {  // the part of the codes inside the word
        const uint64_t s0 = p0 > b0 ? p0 : b0;
        const uint64_t e0 = p0 + plen < b0 + 64 ? p0 + plen : b0 + 64;
        const uint32_t len = (uint32_t)(e0 - s0);
        or_bits(word, b0, (uint64_t)read_bits(pay, pwords, off[L] + (s0 - p0), len), s0, len);
      }
      or_bits(word, b0, 0xffffffffull, p0 + plen, 32);  // end mark
    }
    const bool shared = (w == w_first && (b_beg & 63) && L0 > 0) ||
                        (w == w_last && (b_end & 63) && L0 + cnt < n_leaves);
    if (shared)
      atomicOr((unsigned long long*)&out[w], (unsigned long long)word);
    else
      out[w] = word;
  }
}

hipError_t launch_export(const DecompressPlan& p, const DecompressWs& w, const uint8_t* stream,
                         void* out, uint32_t* d_status, hipStream_t s) {
  BBX_LAUNCH("dec_init", k_dec_init, 1, 64, 0, s, w.params, stream, p.header);
  if (p.n > 0) {
    uint64_t g = (p.n_leaves + kBlock - 1) / kBlock;
    if (g > 65536) g = 65536;
    BBX_LAUNCH("dec_meta", k_dec_meta, g, kBlock, 0, s, p.n_leaves, p.dims, p.mbits, p.G[0],
               p.G[1], p.G[2], p.meta_bits, p.geom, stream, w.leaves, w.leaf_bits, w.params,
               p.ref_mode, p.dtype, p.origin[0], p.origin[1], p.origin[2], p.inv_w);
    hipError_t e = launch_dec_scan(p.n_leaves, w.leaf_bits, w.scan_part, w.params, p.payload_bits, s);
    if (e != hipSuccess) return e;
    const uint32_t M = coord_bits(p.dtype);
    const uint64_t F = (uint64_t)p.dims * (M + p.mbits) + 32;
    const uint64_t blocks = (p.n_leaves + kExportLeaves - 1) / kExportLeaves;
    const uint64_t out_words = (p.n_leaves * F + p.payload_bits + 63) / 64;
    if (blocks > 1)
      BBX_LAUNCH("export_edges", k_export_edges, (blocks - 1 + kBlock - 1) / kBlock, kBlock, 0, s,
                 p.n_leaves, F, w.leaf_bits, (uint64_t*)out, out_words, w.params);
    BBX_LAUNCH("export", k_export, blocks, kBlock, 0, s, p.n_leaves, p.dims, p.mbits, M,
               p.meta_bits, p.payload_bits, w.leaf_bits, stream, (uint64_t*)out, w.params);
  }
  BBX_LAUNCH("dec_finish", k_dec_finish, 1, 64, 0, s, w.params, d_status);
  return hipGetLastError();
}

}  // namespace bbx

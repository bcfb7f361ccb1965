// k_huff.hip -- Huffman coding of a byte buffer: the encoding phase of
// Sec. 3, which the paper applies to its sequence layout (Sec. 4.2).
//
// Symbols are bytes.  Code lengths come from Huffman's construction, the two
// lightest nodes merging first (on equal weights the node created earlier:
// leaves, in symbol order, before merged nodes, in creation order); a tree
// deeper than kHufMaxLen is rebuilt from the weights halved (rounded up)
// until it fits.  Codes are canonical in (length, symbol) order.  The input
// is cut into chunks of kHufChunk bytes whose first bit offsets are stored,
// so that the chunks decode independently.
//
// Stream: [0,4) 'BBXH' | [4,6) version 1 | [6] kHufMaxLen | [7] 0 |
// [8,16) n | [16,20) kHufChunk | [20,24) 0 | [24,32) chunks |
// [32,40) payload bits | [40,48) 0 | [48,176) code lengths, a nibble per
// symbol (low nibble: even symbol) | chunk bit offsets, u64 each, from the
// payload start | payload: the codes in input order, each code's most
// significant bit first, bit i = bit i mod 64 of u64 word i / 64, zero
// padded to 8 bytes.
//
// Encode (the call waits twice: for the histogram, from which the host builds
// the code, and for the total size):
//   k_huf_hist    byte histogram (LDS bins per block, then global atomics)
//   k_huf_count   bits of every chunk (a block per chunk)
//   k_huf_offsets one block: exclusive scan of the chunk bits into the
//                 stream's offset table, and the payload's total bits
//   k_huf_write   a block per chunk: each thread's 64 bytes of codes at its
//                 offset (block scan), ORed into the zeroed payload words
// Decode:
//   k_huf_table   one block: checks the header against the host's copy, the
//                 lengths (at most kHufMaxLen, Kraft sum at most 1), and builds
//                 the 4,096-entry table from a 12-bit window to (symbol, length)
//   k_huf_decode  a thread per chunk, the table in LDS, a 64-bit bit buffer
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "bbx_internal.h"

namespace bbx {

typedef unsigned __int128 u128;

constexpr uint32_t kHufMagic = 0x48584242u;  // bytes 'B','B','X','H'
constexpr uint32_t kHufMaxLen = 12;
constexpr uint32_t kHufChunk = 4096;
constexpr uint32_t kHufHeader = 176;
constexpr uint32_t kHufPer = kHufChunk / kBlock;  // bytes per thread of a chunk block

// The host's copy of a stream header, for the device to compare.
struct HufHeaderCopy {
  uint64_t w[kHufHeader / 8];
};

__host__ __device__ inline uint64_t huf_chunks(uint64_t n) { return (n + kHufChunk - 1) / kHufChunk; }
__host__ __device__ inline uint64_t huf_words(uint64_t bits) { return (bits + 63) / 64; }

// ---------------------------------------------------------------- host: the code

// Code lengths by the two-queue form of Huffman's construction: leaves sorted
// by (weight, symbol) in one queue, merged nodes in creation order in the
// other (their weights never decrease); the lighter front merges first, the
// leaf on equal weights (every leaf was created before every merged node).
static void huf_build_lengths(const uint64_t* counts, uint32_t* len) {
  std::vector<uint64_t> w(counts, counts + 256);
  for (int s = 0; s < 256; ++s) len[s] = 0;
  for (;;) {
    std::vector<int> leaves;
    for (int s = 0; s < 256; ++s)
      if (w[s]) leaves.push_back(s);
    const size_t k = leaves.size();
    if (k == 0) return;
    if (k == 1) {
      len[leaves[0]] = 1;
      return;
    }
    std::stable_sort(leaves.begin(), leaves.end(), [&](int a, int b) { return w[a] < w[b]; });
    // node ids: leaves 0..k-1 (in symbol order), merged k..; parent links
    std::vector<int> leaf_id(256, -1), parent(2 * k - 1, -1);
    {
      int id = 0;
      for (int s = 0; s < 256; ++s)
        if (w[s]) leaf_id[s] = id++;
    }
    std::vector<uint64_t> mw;  // merged nodes' weights, in creation order
    size_t li = 0, mi = 0;
    auto take = [&]() -> std::pair<int, uint64_t> {
      const bool leaf = mi >= mw.size() || (li < k && w[leaves[li]] <= mw[mi]);
      if (leaf) {
        const int s = leaves[li++];
        return {leaf_id[s], w[s]};
      }
      const int id = (int)(k + mi);
      return {id, mw[mi++]};
    };
    for (size_t m = 0; m + 1 < k; ++m) {
      const auto a = take(), b = take();
      const int id = (int)(k + mw.size());
      parent[a.first] = parent[b.first] = id;
      mw.push_back(a.second + b.second);
    }
    uint32_t deepest = 0;
    std::vector<uint32_t> depth(256, 0);
    for (int s = 0; s < 256; ++s) {
      if (!w[s]) continue;
      uint32_t dpt = 0;
      for (int p = parent[leaf_id[s]]; p >= 0; p = parent[p]) ++dpt;
      depth[s] = dpt;
      deepest = std::max(deepest, dpt);
    }
    if (deepest <= kHufMaxLen) {
      for (int s = 0; s < 256; ++s) len[s] = depth[s];
      return;
    }
    for (int s = 0; s < 256; ++s)
      if (w[s]) w[s] = (w[s] + 1) / 2;
  }
}

// Canonical codes, each reversed into the stream's bit order (the code's
// first bit at bit 0), packed with the length: rev | len << 16.
static void huf_build_table(const uint32_t* len, uint32_t* tab) {
  uint32_t code = 0, prev = 0;
  bool first = true;
  for (uint32_t L = 1; L <= kHufMaxLen; ++L)
    for (int s = 0; s < 256; ++s) {
      if (len[s] != L) continue;
      if (!first) code = (code + 1) << (L - prev);
      first = false;
      prev = L;
      uint32_t rev = 0;
      for (uint32_t b = 0; b < L; ++b) rev |= ((code >> (L - 1 - b)) & 1u) << b;
      tab[s] = rev | (L << 16);
    }
  for (int s = 0; s < 256; ++s)
    if (!len[s]) tab[s] = 0;
}

// ---------------------------------------------------------------- kernels

__global__ void __launch_bounds__(kBlock) k_huf_hist(const uint8_t* in, uint64_t n,
                                                     unsigned long long* counts) {
  __shared__ uint32_t h[4][257];  // four copies, staggered across banks
  for (uint32_t i = threadIdx.x; i < 4 * 257; i += kBlock) (&h[0][0])[i] = 0;
  __syncthreads();
  const uint32_t cp = threadIdx.x & 3;
  const uint64_t nv = n / 16;
  const uint4* in4 = (const uint4*)in;
  for (uint64_t v = (uint64_t)blockIdx.x * kBlock + threadIdx.x; v < nv;
       v += (uint64_t)gridDim.x * kBlock) {
    const uint4 q = in4[v];
    const uint32_t wv[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int b = 0; b < 4; ++b) atomicAdd(&h[cp][(wv[k] >> (8 * b)) & 255u], 1u);
  }
  if (blockIdx.x == 0)
    for (uint64_t i = nv * 16 + threadIdx.x; i < n; i += kBlock) atomicAdd(&h[cp][in[i]], 1u);
  __syncthreads();
  const uint32_t c = h[0][threadIdx.x] + h[1][threadIdx.x] + h[2][threadIdx.x] + h[3][threadIdx.x];
  if (c) atomicAdd(&counts[threadIdx.x], (unsigned long long)c);
}

__device__ inline uint64_t huf_block_exscan(uint64_t v, uint64_t* total) {
  __shared__ uint64_t ws[16];
  const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  uint64_t x = v;
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t y = __shfl_up(x, o);
    if ((int)lane >= o) x += y;
  }
  if (lane == 63) ws[wv] = x;
  __syncthreads();
  uint64_t off = 0, tot = 0;
  for (uint32_t k = 0; k < nw; ++k) {
    off += k < wv ? ws[k] : 0ull;
    tot += ws[k];
  }
  __syncthreads();
  *total = tot;
  return off + x - v;
}

// bits of the thread's bytes [c * kHufChunk + t * kHufPer, ...) of chunk c
__device__ inline uint64_t huf_thread_bits(const uint8_t* in, uint64_t n, uint64_t a,
                                           const uint32_t* tab) {
  uint64_t b = 0;
  for (uint32_t k = 0; k < kHufPer; ++k)
    if (a + k < n) b += tab[in[a + k]] >> 16;
  return b;
}

__global__ void __launch_bounds__(kBlock) k_huf_count(const uint8_t* in, uint64_t n,
                                                      const uint32_t* tab0, uint64_t* chunk_bits) {
  __shared__ uint32_t tab[256];
  tab[threadIdx.x] = tab0[threadIdx.x];
  __syncthreads();
  const uint64_t a = (uint64_t)blockIdx.x * kHufChunk + (uint64_t)threadIdx.x * kHufPer;
  uint64_t tot;
  huf_block_exscan(huf_thread_bits(in, n, a, tab), &tot);
  if (threadIdx.x == 0) chunk_bits[blockIdx.x] = tot;
}

// One block: chunk offsets into the stream (after the header) and the total.
__global__ void __launch_bounds__(1024) k_huf_offsets(const uint64_t* chunk_bits, uint64_t chunks,
                                                      uint8_t* out, uint64_t* total_out) {
  uint64_t* offs = (uint64_t*)(out + kHufHeader);
  uint64_t run = 0;
  for (uint64_t c0 = 0; c0 < chunks; c0 += blockDim.x) {
    const uint64_t c = c0 + threadIdx.x;
    const uint64_t v = c < chunks ? chunk_bits[c] : 0ull;
    uint64_t tot;
    const uint64_t ex = huf_block_exscan(v, &tot);
    if (c < chunks) offs[c] = run + ex;
    run += tot;
  }
  if (threadIdx.x == 0) {
    *total_out = run;
    *(uint64_t*)(out + 32) = run;  // payload bits
  }
}

__global__ void __launch_bounds__(kBlock) k_huf_zero(uint64_t* p, uint64_t words) {
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < words;
       i += (uint64_t)gridDim.x * kBlock)
    p[i] = 0;
}

__global__ void __launch_bounds__(kBlock) k_huf_write(const uint8_t* in, uint64_t n,
                                                      const uint32_t* tab0, uint8_t* out,
                                                      uint64_t chunks) {
  __shared__ uint32_t tab[256];
  tab[threadIdx.x] = tab0[threadIdx.x];
  __syncthreads();
  const uint64_t c = blockIdx.x;
  const uint64_t* offs = (const uint64_t*)(out + kHufHeader);
  unsigned long long* pay = (unsigned long long*)(out + kHufHeader + 8 * chunks);
  const uint64_t a = c * kHufChunk + (uint64_t)threadIdx.x * kHufPer;
  uint64_t tot;
  uint64_t pos = offs[c] + huf_block_exscan(huf_thread_bits(in, n, a, tab), &tot);
  // the thread's codes gathered in a 64-bit window; a full word (or the
  // last, partial one) is ORed into the payload
  uint64_t win = 0;
  uint32_t fill = (uint32_t)(pos & 63);
  uint64_t word = pos >> 6;
  for (uint32_t k = 0; k < kHufPer; ++k) {
    if (a + k >= n) break;
    const uint32_t e = tab[in[a + k]];
    const uint32_t L = e >> 16;
    const uint64_t rev = e & 0xffffu;
    win |= rev << fill;
    if (fill + L >= 64) {
      atomicOr(&pay[word], (unsigned long long)win);
      const uint32_t used = 64 - fill;  // bits of this code that went into the word
      win = used < 64 ? rev >> used : 0ull;
      fill = fill + L - 64;
      ++word;
    } else {
      fill += L;
    }
  }
  if (fill > 0) atomicOr(&pay[word], (unsigned long long)win);
}

// Decode table: 12-bit window (the code's first bit at bit 0) -> symbol |
// length << 8, 0 where no code matches.  Also checks the stream's header
// against the host's copy and the lengths.
__global__ void __launch_bounds__(kBlock) k_huf_table(const uint8_t* s, HufHeaderCopy h,
                                                      uint16_t* table, uint32_t* status) {
  __shared__ uint32_t tab[256];
  __shared__ uint32_t bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < kHufHeader / 8; i += kBlock)
    if (((const uint64_t*)s)[i] != h.w[i]) atomicOr(&bad, 1u);
  __syncthreads();
  if (threadIdx.x == 0 && !bad) {
    uint32_t len[256];
    uint64_t kraft = 0;
    for (int t = 0; t < 256; ++t) {
      len[t] = (s[48 + t / 2] >> ((t & 1) ? 4 : 0)) & 15u;
      if (len[t] > kHufMaxLen) bad = 1;
      if (len[t]) kraft += 1ull << (kHufMaxLen - len[t]);
    }
    if (kraft > (1ull << kHufMaxLen)) bad = 1;
    uint32_t code = 0, prev = 0;
    bool first = true;
    for (uint32_t L = 1; L <= kHufMaxLen && !bad; ++L)
      for (int t = 0; t < 256; ++t) {
        if (len[t] != L) continue;
        if (!first) code = (code + 1) << (L - prev);
        first = false;
        prev = L;
        uint32_t rev = 0;
        for (uint32_t b = 0; b < L; ++b) rev |= ((code >> (L - 1 - b)) & 1u) << b;
        tab[t] = rev | (L << 16);
      }
    for (int t = 0; t < 256; ++t)
      if (!len[t]) tab[t] = 0;
  }
  __syncthreads();
  if (bad) {
    if (threadIdx.x == 0) *status = BBX_ECORRUPT;
    return;
  }
  for (uint32_t x = threadIdx.x; x < (1u << kHufMaxLen); x += kBlock) table[x] = 0;
  __syncthreads();
  for (uint32_t t = 0; t < 256; ++t) {
    const uint32_t e = tab[t], L = e >> 16;
    if (!L) continue;
    const uint32_t rev = e & 0xffffu;
    for (uint32_t hi = threadIdx.x; hi < (1u << (kHufMaxLen - L)); hi += kBlock)
      table[rev | (hi << L)] = (uint16_t)(t | (L << 8));
  }
}

__global__ void __launch_bounds__(kBlock) k_huf_decode(const uint8_t* s, uint64_t n, uint64_t chunks,
                                                       uint64_t bits, const uint16_t* table0,
                                                       uint8_t* out, uint32_t* status) {
  __shared__ uint16_t table[1u << kHufMaxLen];
  if (*status != BBX_OK) return;
  for (uint32_t x = threadIdx.x; x < (1u << kHufMaxLen); x += kBlock) table[x] = table0[x];
  __syncthreads();
  const uint64_t c = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (c >= chunks) return;
  const uint64_t* offs = (const uint64_t*)(s + kHufHeader);
  const uint64_t* pay = offs + chunks;
  const uint64_t nwords = huf_words(bits);
  uint64_t pos = offs[c];
  const uint64_t end = c + 1 < chunks ? offs[c + 1] : bits;
  if (pos > end || end > bits) {
    atomicExch(status, (uint32_t)BBX_ECORRUPT);
    return;
  }
  const uint64_t i0 = c * kHufChunk, i1 = i0 + kHufChunk < n ? i0 + kHufChunk : n;
  // bit reader: `acc` holds the stream's bits [pos, pos + have); the next
  // word is loaded one refill ahead, so its latency overlaps the decoding of
  // the bits before it
  uint64_t wd = pos >> 6;
  const uint32_t sh0 = (uint32_t)(pos & 63);
  u128 acc = wd < nwords ? (u128)(pay[wd] >> sh0) : (u128)0;
  uint32_t have = 64 - sh0;
  ++wd;
  uint64_t next = wd < nwords ? pay[wd] : 0ull;
  ++wd;
  uint64_t pk = 0;  // eight decoded bytes, stored together
  for (uint64_t i = i0; i < i1; ++i) {
    if (have < 64) {
      acc |= (u128)next << have;
      have += 64;
      next = wd < nwords ? pay[wd] : 0ull;
      ++wd;
    }
    const uint64_t buf = (uint64_t)acc;
    const uint16_t e = table[buf & ((1u << kHufMaxLen) - 1)];
    const uint32_t L = e >> 8;
    if (L == 0 || pos + L > end) {
      atomicExch(status, (uint32_t)BBX_ECORRUPT);
      return;
    }
    pk |= (uint64_t)(e & 0xffu) << (8 * (i & 7));
    if ((i & 7) == 7 || i + 1 == i1) {
      const uint64_t b0 = i & ~(uint64_t)7;
      if ((i & 7) == 7)
        *(uint64_t*)(out + b0) = pk;
      else
        for (uint64_t t = b0; t <= i; ++t) out[t] = (uint8_t)(pk >> (8 * (t - b0)));
      pk = 0;
    }
    acc >>= L;
    have -= L;
    pos += L;
  }
  if (pos != end) atomicExch(status, (uint32_t)BBX_ECORRUPT);
}

}  // namespace bbx

using namespace bbx;

namespace {

struct HufHead {
  uint64_t n, chunks, bits;
};

bbx_status huf_parse(const uint8_t* h, size_t bytes, HufHead* o) {
  if (!h || bytes < kHufHeader) return set_error(BBX_ECORRUPT, "Huffman stream shorter than its header");
  uint32_t magic, chunk;
  uint16_t ver;
  memcpy(&magic, h, 4);
  memcpy(&ver, h + 4, 2);
  memcpy(&chunk, h + 16, 4);
  memcpy(&o->n, h + 8, 8);
  memcpy(&o->chunks, h + 24, 8);
  memcpy(&o->bits, h + 32, 8);
  uint64_t z0, z1 = 0;
  memcpy(&z0, h + 40, 8);
  memcpy(&z1, h + 20, 4);
  if (magic != kHufMagic || ver != 1 || h[6] != kHufMaxLen || h[7] != 0 || chunk != kHufChunk ||
      z0 != 0 || z1 != 0)
    return set_error(BBX_ECORRUPT, "not a Huffman stream of this version");
  if (o->chunks != huf_chunks(o->n) || o->bits > o->n * kHufMaxLen)
    return set_error(BBX_ECORRUPT, "Huffman chunk count or payload size out of range");
  return BBX_OK;
}

size_t huf_decode_ws(uint64_t chunks) {
  (void)chunks;
  return 256 + 2 * (1u << kHufMaxLen);
}

}  // namespace

extern "C" {

size_t bbx_huffman_bound(uint64_t n) {
  return kHufHeader + 8 * huf_chunks(n) + 8 * huf_words(n * kHufMaxLen);
}

size_t bbx_huffman_workspace_size(uint64_t n) {
  // counts (256 u64), code table (256 u32), chunk bits (u64 each), the total,
  // or when decoding: status and the 4,096-entry table
  const size_t enc = 2048 + 1024 + 8 * huf_chunks(n) + 8 + 256;
  return std::max(enc, huf_decode_ws(huf_chunks(n)));
}

bbx_status bbx_huffman_encode(const void* d_in, uint64_t n, void* d_out, size_t out_cap,
                              size_t* h_out_size, void* d_ws, size_t ws_size, hipStream_t stream) {
  if (!h_out_size) return set_error(BBX_EINVAL, "h_out_size is NULL");
  if (n > 0 && !d_in) return set_error(BBX_EINVAL, "input pointer is NULL");
  if (!d_out || ((uintptr_t)d_out & 7)) return set_error(BBX_EINVAL, "output must be 8-byte aligned");
  if (((uintptr_t)d_in & 15) && n >= 16) return set_error(BBX_EINVAL, "input must be 16-byte aligned");
  if (!d_ws || ((uintptr_t)d_ws & 255) || ws_size < bbx_huffman_workspace_size(n))
    return set_error(BBX_ENOMEM, "workspace too small or not 256-byte aligned");
  const uint64_t chunks = huf_chunks(n);
  uint8_t* ws = (uint8_t*)d_ws;
  unsigned long long* counts = (unsigned long long*)ws;
  uint32_t* tab = (uint32_t*)(ws + 2048);
  uint64_t* cbits = (uint64_t*)(ws + 3072);
  uint64_t* total = cbits + chunks;
  const uint8_t* in = (const uint8_t*)d_in;
  uint8_t* out = (uint8_t*)d_out;
  hipError_t e = hipMemsetAsync(counts, 0, 2048, stream);
  if (e == hipSuccess && n > 0)
    BBX_LAUNCH("huf_hist", k_huf_hist, (uint32_t)std::min<uint64_t>((n / 16 + kBlock - 1) / kBlock + 1, 2048),
               kBlock, 0, stream, in, n, counts);
  uint64_t hc[256];
  if (e == hipSuccess) e = hipMemcpyAsync(hc, counts, sizeof(hc), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return set_error(BBX_EHIP, hipGetErrorString(e));
  uint32_t len[256], htab[256];
  huf_build_lengths(hc, len);
  huf_build_table(len, htab);
  uint64_t bits = 0;
  for (int s = 0; s < 256; ++s) bits += hc[s] * len[s];
  const size_t size = kHufHeader + 8 * chunks + 8 * huf_words(bits);
  *h_out_size = size;
  if (size > out_cap) return set_error(BBX_ENOSPC, "output capacity below the Huffman stream");
  uint8_t head[kHufHeader];
  memset(head, 0, sizeof(head));
  const uint32_t magic = kHufMagic, chunk = kHufChunk;
  const uint16_t ver = 1;
  memcpy(head, &magic, 4);
  memcpy(head + 4, &ver, 2);
  head[6] = (uint8_t)kHufMaxLen;
  memcpy(head + 8, &n, 8);
  memcpy(head + 16, &chunk, 4);
  memcpy(head + 24, &chunks, 8);
  memcpy(head + 32, &bits, 8);
  for (int s = 0; s < 256; ++s) head[48 + s / 2] |= (uint8_t)(len[s] << ((s & 1) ? 4 : 0));
  e = hipMemcpyAsync(out, head, kHufHeader, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipMemcpyAsync(tab, htab, sizeof(htab), hipMemcpyHostToDevice, stream);
  if (e == hipSuccess && chunks > 0) {
    BBX_LAUNCH("huf_count", k_huf_count, (uint32_t)chunks, kBlock, 0, stream, in, n, tab, cbits);
    BBX_LAUNCH("huf_offsets", k_huf_offsets, 1, 1024, 0, stream, cbits, chunks, out, total);
    BBX_LAUNCH("huf_zero", k_huf_zero, (uint32_t)std::min<uint64_t>(huf_words(bits) / kBlock + 1, 4096),
               kBlock, 0, stream, (uint64_t*)(out + kHufHeader + 8 * chunks), huf_words(bits));
    BBX_LAUNCH("huf_write", k_huf_write, (uint32_t)chunks, kBlock, 0, stream, in, n, tab, out, chunks);
    e = hipGetLastError();
  }
  uint64_t dev_bits = bits;
  if (e == hipSuccess && chunks > 0)
    e = hipMemcpyAsync(&dev_bits, total, 8, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return set_error(BBX_EHIP, hipGetErrorString(e));
  if (dev_bits != bits) return set_error(BBX_EHIP, "chunk bit counts disagree with the histogram");
  return BBX_OK;
}

bbx_status bbx_huffman_decode(const void* d_stream, size_t stream_size, const void* h_header,
                              void* d_out, size_t out_cap, uint32_t* d_status, void* d_ws,
                              size_t ws_size, hipStream_t stream) {
  HufHead h;
  bbx_status st = huf_parse((const uint8_t*)h_header, h_header ? kHufHeader : 0, &h);
  if (st != BBX_OK) return st;
  if (!d_stream || stream_size < kHufHeader + 8 * h.chunks + 8 * huf_words(h.bits))
    return set_error(BBX_ECORRUPT, "Huffman stream shorter than its sections");
  if (h.n > out_cap) return set_error(BBX_ENOSPC, "output capacity below the decoded size");
  if (h.n > 0 && (!d_out || ((uintptr_t)d_out & 7))) return set_error(BBX_EINVAL, "output must be 8-byte aligned");
  if (!d_ws || ((uintptr_t)d_ws & 255) || ws_size < huf_decode_ws(h.chunks))
    return set_error(BBX_ENOMEM, "workspace too small or not 256-byte aligned");
  uint8_t* ws = (uint8_t*)d_ws;
  uint32_t* status = d_status ? d_status : (uint32_t*)ws;
  uint16_t* table = (uint16_t*)(ws + 256);
  HufHeaderCopy hc;
  memcpy(hc.w, h_header, kHufHeader);
  hipError_t e = hipMemsetAsync(status, 0, 4, stream);
  if (e == hipSuccess) {
    BBX_LAUNCH("huf_table", k_huf_table, 1, kBlock, 0, stream, (const uint8_t*)d_stream, hc, table,
               status);
    if (h.chunks > 0)
      BBX_LAUNCH("huf_decode", k_huf_decode, (uint32_t)((h.chunks + kBlock - 1) / kBlock), kBlock, 0,
                 stream, (const uint8_t*)d_stream, h.n, h.chunks, h.bits, table, (uint8_t*)d_out,
                 status);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return set_error(BBX_EHIP, hipGetErrorString(e));
  if (d_status) return BBX_OK;
  uint32_t hs = 0;
  e = hipMemcpyAsync(&hs, status, 4, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return set_error(BBX_EHIP, hipGetErrorString(e));
  if (hs != BBX_OK) return set_error((bbx_status)hs, "the Huffman stream fails validation");
  return BBX_OK;
}

}  // extern "C"

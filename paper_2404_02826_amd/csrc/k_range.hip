// k_range.hip -- range and bound (Sec. 3) and quantization (Sec. 3,
// linear-scale quantization into bins of width 2*eb), for every set of a batch.
//
//   k_minmax    per-block per-axis min/max + non-finite flag (one HBM read)
//   k_epilogue  one block per set: reduces the partials and computes, in FP64
//               with one rounding per operation, Delta_max, eb_abs, the
//               rounding guard, eb_eff, w = 2*eb_eff, inv_w and the code
//               widths G_d
//   k_quantize  q = floor((x - lo) * inv_w + 1/2) per coordinate, written as
//               structure-of-arrays codes (u16 when every G_d <= 16, else u32);
//               also the depth-0 first-digit histogram of the k-d partition
#include <math.h>

#include <type_traits>

#include "bbx_internal.h"

namespace bbx {

template <typename T>
__device__ inline double load_coord(const T* pos, uint64_t n, uint32_t dims, uint32_t layout,
                                    uint64_t i, uint32_t d) {
  return (double)(layout == BBX_AOS ? pos[i * dims + d] : pos[(uint64_t)d * n + i]);
}

__device__ inline double wave_min(double v) {
  for (int o = 32; o > 0; o >>= 1) {
    double u = __shfl_xor(v, o);
    v = u < v ? u : v;
  }
  return v;
}
__device__ inline double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) {
    double u = __shfl_xor(v, o);
    v = u > v ? u : v;
  }
  return v;
}

// Array-of-structures input with a 16-byte aligned base: a thread reads V
// consecutive particles (DIMS 16-byte loads) at a time, so each loaded
// element's axis is fixed; the remaining particles go one by one.
template <typename T, int DIMS>
__device__ uint64_t minmax_aos_vec(const T* __restrict__ pos, uint64_t n, uint64_t t0, uint64_t nt,
                                   double* lo, double* hi, double& bad) {
  constexpr uint32_t V = 16 / sizeof(T);
  const uint64_t ng = n / V;
  const uint4* p4 = (const uint4*)pos;
  for (uint64_t g = t0; g < ng; g += nt) {
    union {
      uint4 v[DIMS];
      T e[DIMS * V];
    } u;
#pragma unroll
    for (int i = 0; i < DIMS; ++i) u.v[i] = p4[g * DIMS + i];
#pragma unroll
    for (int e = 0; e < DIMS * (int)V; ++e) {
      const int d = e % DIMS;
      const double v = (double)u.e[e];
      if (!isfinite(v)) bad = 1.0;
      lo[d] = v < lo[d] ? v : lo[d];
      hi[d] = v > hi[d] ? v : hi[d];
    }
  }
  return ng * V;  // particles handled
}

template <typename T>
__device__ void minmax_body(const T* __restrict__ pos, uint64_t n, uint32_t dims, uint32_t layout,
                            uint64_t lb, uint32_t mm_blocks, double* part) {
  double lo[3] = {INFINITY, INFINITY, INFINITY};
  double hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  double bad = 0.0;
  const uint64_t stride = (uint64_t)mm_blocks * blockDim.x;
  uint64_t first = 0;
  if (layout == BBX_AOS && ((uintptr_t)pos & 15) == 0)
    first = dims == 3 ? minmax_aos_vec<T, 3>(pos, n, lb * blockDim.x + threadIdx.x, stride, lo, hi, bad)
                      : minmax_aos_vec<T, 2>(pos, n, lb * blockDim.x + threadIdx.x, stride, lo, hi, bad);
  for (uint64_t i = first + lb * blockDim.x + threadIdx.x; i < n; i += stride) {
#pragma unroll
    for (uint32_t d = 0; d < 3; ++d) {
      if (d >= dims) break;
      const double v = load_coord(pos, n, dims, layout, i, d);
      if (!isfinite(v)) bad = 1.0;
      lo[d] = v < lo[d] ? v : lo[d];
      hi[d] = v > hi[d] ? v : hi[d];
    }
  }
  __shared__ double sh[8][kBlock / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int d = 0; d < 3; ++d) {
    const double a = wave_min(lo[d]), b = wave_max(hi[d]);
    if (lane == 0) sh[d][wv] = a, sh[3 + d][wv] = b;
  }
  const double bb = wave_max(bad);
  if (lane == 0) sh[6][wv] = bb;
  __syncthreads();
  if (threadIdx.x < 7) {
    const int f = threadIdx.x;
    double v = sh[f][0];
    for (int k = 1; k < kBlock / 64; ++k) {
      const double u = sh[f][k];
      if (f < 3)
        v = u < v ? u : v;
      else
        v = u > v ? u : v;
    }
    part[f] = v;
  }
}

// partials layout per block: lo[3], hi[3], bad, unused (8 doubles)
__global__ void __launch_bounds__(kBlock) k_minmax(uint32_t nsets, const uint64_t* pre,
                                                   const SetDesc* sets, double* partials) {
  const uint32_t s = find_set(pre, nsets, blockIdx.x);
  const SetDesc& S = sets[s];
  const uint64_t lb = blockIdx.x - pre[s];
  double* part = partials + (S.part_off + lb) * 8;
  const uint64_t n = S.n;
  const uint32_t dims = S.dims, layout = S.layout, mmb = S.mm_blocks;
  if (S.dtype == BBX_F32)
    minmax_body<float>((const float*)S.pos, n, dims, layout, lb, mmb, part);
  else
    minmax_body<double>((const double*)S.pos, n, dims, layout, lb, mmb, part);
}

__global__ void __launch_bounds__(kBlock) k_epilogue(const SetDesc* sets, const double* partials,
                                                     DevParams* params) {
  const SetDesc& S = sets[blockIdx.x];
  DevParams* P = params + blockIdx.x;
  __shared__ double red[7][kBlock / 64];
  double v[7];
  for (int f = 0; f < 7; ++f) v[f] = f < 3 ? INFINITY : (f < 6 ? -INFINITY : 0.0);
  for (uint32_t b = threadIdx.x; b < S.mm_blocks; b += blockDim.x)
    for (int f = 0; f < 7; ++f) {
      const double u = partials[(S.part_off + b) * 8 + f];
      if (f < 3)
        v[f] = u < v[f] ? u : v[f];
      else
        v[f] = u > v[f] ? u : v[f];
    }
  // min / max are exact in any order: wavefront reductions, then the four
  // wavefront results
  for (int f = 0; f < 7; ++f) v[f] = f < 3 ? wave_min(v[f]) : wave_max(v[f]);
  if ((threadIdx.x & 63) == 0)
    for (int f = 0; f < 7; ++f) red[f][threadIdx.x >> 6] = v[f];
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int f = 0; f < 7; ++f)
    for (int t = 1; t < kBlock / 64; ++t) {
      const double u = red[f][t];
      if (f < 3)
        v[f] = u < v[f] ? u : v[f];
      else
        v[f] = u > v[f] ? u : v[f];
    }

  const uint64_t n = S.n;
  const uint32_t dims = S.dims;
  const double eb = S.eb;
  DevParams p;
  for (int d = 0; d < 3; ++d) p.lo[d] = p.hi[d] = 0.0, p.G[d] = 0;
  p.eb_user = eb;
  p.eb_abs = p.eb_eff = p.w = p.inv_w = 0.0;
  p.key16 = 1;
  p.status = BBX_OK;
  p.diag = 0;
  p.meta_bits = p.payload_bits = p.total_bytes = p.payload_base = 0;
  p.nseq = 0;
  p.nleaves = 0;
  p.pad1[0] = 0;
  if (n == 0) {
    p.eb_abs = S.eb_mode == BBX_EB_ABS ? eb : 0.0;
    *P = p;
    return;
  }
  if (v[6] != 0.0) {
    p.status = BBX_EINVAL;  // NaN or Inf coordinate
    *P = p;
    return;
  }
  for (uint32_t d = 0; d < dims; ++d) {
    p.lo[d] = v[d] + 0.0;  // -0.0 becomes +0.0
    p.hi[d] = v[3 + d] + 0.0;
  }
  double delta = 0.0;
  for (uint32_t d = 0; d < dims; ++d) {
    const double rg = p.hi[d] - p.lo[d];
    if (rg > delta) delta = rg;
  }
  p.eb_abs = S.eb_mode == BBX_EB_REL ? eb * delta : eb;
  if (!isfinite(delta) || !isfinite(p.eb_abs)) {
    p.status = kStatusLossless;  // the grid cannot meet the bound
    *P = p;
    return;
  }
  if (delta != 0.0) {
    double amax = 0.0;
    for (uint32_t d = 0; d < dims; ++d) {
      const double a = fabs(p.lo[d]) > fabs(p.hi[d]) ? fabs(p.lo[d]) : fabs(p.hi[d]);
      if (a > amax) amax = a;
    }
    amax = amax + p.eb_abs;
    double guard = ldexp(amax, -48);
    if (S.dtype == BBX_F32) {
      int e = 0;
      (void)frexp(amax, &e);
      double half_ulp = ldexp(1.0, e - 25);
      const double tiny = ldexp(1.0, -150);
      if (half_ulp < tiny) half_ulp = tiny;
      guard = guard + half_ulp;
    }
    p.eb_eff = p.eb_abs - guard;
    if (!(p.eb_eff > 0.0)) {
      p.status = kStatusLossless;
      *P = p;
      return;
    }
    p.w = 2.0 * p.eb_eff;
    p.inv_w = 1.0 / p.w;
    if (!isfinite(p.w) || !isfinite(p.inv_w) || !(p.inv_w > 0.0)) {
      p.status = kStatusLossless;
      *P = p;
      return;
    }
    for (uint32_t d = 0; d < dims; ++d) {
      const double qm = floor((p.hi[d] - p.lo[d]) * p.inv_w + 0.5);
      if (!(qm < 1073741824.0)) {
        p.status = kStatusLossless;  // codes of 30 bits or more
        *P = p;
        return;
      }
      p.G[d] = bitlen32((uint32_t)qm);
      if (p.G[d] > 16) p.key16 = 0;
    }
  }
  *P = p;
}

// Root histogram: when the depth-0 median is selected with global histograms,
// quantization also counts the first radix digit of every axis-0 code into
// the block's LDS bins (lh != null), so that level needs no pass of its own.
template <typename T, typename KT, int DIMS>
__device__ uint64_t quantize_aos_vec(const T* __restrict__ pos, uint64_t n, uint64_t kst,
                                     const double* lo, double inv_w, uint64_t t0, uint64_t nt,
                                     KT* __restrict__ keys, uint32_t* __restrict__ idx,
                                     uint32_t* lh, uint32_t hsh, uint32_t hmask) {
  constexpr uint32_t V = 16 / sizeof(T);  // particles per group (2 or 4)
  const uint64_t ng = n / V;
  const uint4* p4 = (const uint4*)pos;
  for (uint64_t g = t0; g < ng; g += nt) {
    union {
      uint4 v[DIMS];
      T e[DIMS * V];
    } u;
#pragma unroll
    for (int i = 0; i < DIMS; ++i) u.v[i] = p4[g * DIMS + i];
#pragma unroll
    for (int d = 0; d < DIMS; ++d) {
      union {
        KT k[V];
        typename std::conditional<sizeof(KT) * V == 16, uint4,
                 typename std::conditional<sizeof(KT) * V == 8, uint2, uint32_t>::type>::type w;
      } o;
#pragma unroll
      for (uint32_t j = 0; j < V; ++j) {
        const uint32_t q = (uint32_t)floor(((double)u.e[j * DIMS + d] - lo[d]) * inv_w + 0.5);
        o.k[j] = (KT)q;
        if (d == 0 && lh) atomicAdd(&lh[(q >> hsh) & hmask], 1u);
      }
      *(decltype(o.w)*)(keys + (uint64_t)d * kst + g * V) = o.w;
    }
    if (idx)
#pragma unroll
      for (uint32_t j = 0; j < V; ++j) idx[g * V + j] = (uint32_t)(g * V + j);
  }
  return ng * V;
}

template <typename T, typename KT>
__device__ void quantize_body(const T* __restrict__ pos, uint64_t n, uint64_t kst, uint32_t dims,
                              uint32_t layout, double lo0, double lo1, double lo2, double inv_w,
                              uint64_t lb, uint64_t nblk, KT* __restrict__ keys,
                              uint32_t* __restrict__ idx, uint32_t* lh, uint32_t hsh,
                              uint32_t hmask) {
  const double lo[3] = {lo0, lo1, lo2};
  const uint64_t stride = nblk * blockDim.x;
  uint64_t first = 0;
  if (layout == BBX_AOS && ((uintptr_t)pos & 15) == 0)
    first = dims == 3 ? quantize_aos_vec<T, KT, 3>(pos, n, kst, lo, inv_w, lb * blockDim.x + threadIdx.x,
                                                   stride, keys, idx, lh, hsh, hmask)
                      : quantize_aos_vec<T, KT, 2>(pos, n, kst, lo, inv_w, lb * blockDim.x + threadIdx.x,
                                                   stride, keys, idx, lh, hsh, hmask);
  for (uint64_t i = first + lb * blockDim.x + threadIdx.x; i < n; i += stride) {
#pragma unroll
    for (uint32_t d = 0; d < 3; ++d) {
      if (d >= dims) break;
      const double x = load_coord(pos, n, dims, layout, i, d);
      const uint32_t q = (uint32_t)floor((x - lo[d]) * inv_w + 0.5);
      keys[(uint64_t)d * kst + i] = (KT)q;
      if (d == 0 && lh) atomicAdd(&lh[(q >> hsh) & hmask], 1u);
    }
    if (idx) idx[i] = (uint32_t)i;
  }
}

template <typename T>
__device__ void quantize_set(const SetDesc& S, const DevParams* P, uint64_t lb, uint64_t nblk,
                             uint8_t* keys, uint32_t* idx, uint32_t* lh, uint32_t hsh,
                             uint32_t hmask) {
  const T* pos = (const T*)S.pos;
  const uint64_t n = S.n;
  const uint32_t dims = S.dims, layout = S.layout;
  const double l0 = P->lo[0], l1 = P->lo[1], l2 = P->lo[2], iw = P->inv_w;
  if (P->key16)
    quantize_body<T, uint16_t>(pos, n, S.kst, dims, layout, l0, l1, l2, iw, lb, nblk,
                               (uint16_t*)keys, idx, lh, hsh, hmask);
  else
    quantize_body<T, uint32_t>(pos, n, S.kst, dims, layout, l0, l1, l2, iw, lb, nblk,
                               (uint32_t*)keys, idx, lh, hsh, hmask);
}

__global__ void __launch_bounds__(kBlock) k_quantize(uint32_t nsets, const uint64_t* pre,
                                                     const SetDesc* sets, const DevParams* params,
                                                     uint8_t* keys0, uint32_t* idx0,
                                                     uint32_t* hist0) {
  const uint32_t s = find_set(pre, nsets, blockIdx.x);
  const SetDesc& S = sets[s];
  const DevParams* P = params + s;
  if (P->status != BBX_OK) return;
  const uint64_t lb = blockIdx.x - pre[s], nblk = pre[s + 1] - pre[s];
  uint32_t* idx = S.track ? idx0 + S.idx_off : nullptr;
  // the depth-0 first-digit histogram, when depth 0 uses global histograms
  // with more than one digit pass (the same condition the level kernels use)
  __shared__ uint32_t lh[kHistBins];
  const DigitPlan pl = digit_plan(P->G[0]);
  const bool root = !S.split && !level_is_local(S.n, 0) && !level_fused(S, 0) && pl.npass >= 2 && S.n > S.r;
  const uint32_t hsh = pl.shift[0], hmask = (1u << pl.width[0]) - 1;
  if (root) {
    lh[threadIdx.x] = 0;
    __syncthreads();
  }
  if (S.dtype == BBX_F32)
    quantize_set<float>(S, P, lb, nblk, keys0 + S.key_off, idx, root ? lh : nullptr, hsh, hmask);
  else
    quantize_set<double>(S, P, lb, nblk, keys0 + S.key_off, idx, root ? lh : nullptr, hsh, hmask);
  if (root) {
    __syncthreads();
    if (threadIdx.x <= hmask && lh[threadIdx.x])
      atomicAdd(&hist0[S.hist_off + threadIdx.x], lh[threadIdx.x]);
  }
}

__global__ void __launch_bounds__(kBlock) k_hist_zero(uint64_t entries, uint32_t* hist) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < entries;
       i += (uint64_t)gridDim.x * blockDim.x)
    hist[i] = 0;
}

hipError_t launch_range(const BatchPlan& bp, const Ws& w, hipStream_t s) {
  if (bp.g_mm > 0)
    BBX_LAUNCH("range_minmax", k_minmax, bp.g_mm, kBlock, 0, s, bp.nsets, w.pre + bp.o_mm, w.sets,
               w.partials);
  BBX_LAUNCH("range_epilogue", k_epilogue, bp.nsets, kBlock, 0, s, w.sets, w.partials, w.params);
  // histogram bins start at zero (the quantize pass adds the root histogram;
  // every select kernel re-zeroes the bins it reads)
  if (bp.hist_entries > 0)
    BBX_LAUNCH("level_hist_zero", k_hist_zero, 1024, kBlock, 0, s, bp.hist_entries, w.hist);
  BBX_LAUNCH("lossless_zero", k_hist_zero, 1, 64, 0, s, (uint64_t)1, w.lossless);  // list count
  if (bp.g_qz > 0)
    BBX_LAUNCH("quantize", k_quantize, bp.g_qz, kBlock, 0, s, bp.nsets, w.pre + bp.o_qz, w.sets,
               w.params, w.keys[0], w.idx[0], w.hist);
  return hipGetLastError();
}

}  // namespace bbx

// k_range.hip -- range and bound (Sec. 3) and quantization (Sec. 3,
// linear-scale quantization into bins of width 2*eb).
//
//   k_minmax    per-block per-axis min/max + non-finite flag (one HBM read)
//   k_epilogue  one block: reduces the partials and computes, in FP64 with
//               one rounding per operation, Delta_max, eb_abs, the rounding
//               guard, eb_eff, w = 2*eb_eff, inv_w and the code widths G_d
//   k_quantize  q = floor((x - lo) * inv_w + 1/2) per coordinate, written as
//               structure-of-arrays keys (u16 when every G_d <= 16, else u32)
#include <math.h>

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

// partials layout per block: lo[3], hi[3], bad, count (8 doubles)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_minmax(const T* pos, uint64_t n, uint32_t dims,
                                                   uint32_t layout, double* partials) {
  double lo[3] = {INFINITY, INFINITY, INFINITY};
  double hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  double bad = 0.0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    for (uint32_t d = 0; d < dims; ++d) {
      double v = load_coord(pos, n, dims, layout, i, d);
      if (!isfinite(v)) bad = 1.0;
      lo[d] = v < lo[d] ? v : lo[d];
      hi[d] = v > hi[d] ? v : hi[d];
    }
  }
  __shared__ double sh[8][kBlock / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int d = 0; d < 3; ++d) {
    double a = wave_min(lo[d]), b = wave_max(hi[d]);
    if (lane == 0) sh[d][wv] = a, sh[3 + d][wv] = b;
  }
  double bb = wave_max(bad);
  if (lane == 0) sh[6][wv] = bb;
  __syncthreads();
  if (threadIdx.x < 7) {
    int f = threadIdx.x;
    double v = sh[f][0];
    for (int k = 1; k < kBlock / 64; ++k) {
      double u = sh[f][k];
      if (f < 3)
        v = u < v ? u : v;
      else
        v = u > v ? u : v;
    }
    partials[blockIdx.x * 8 + f] = v;
  }
}

__global__ void __launch_bounds__(kBlock) k_epilogue(const double* partials, uint32_t nparts,
                                                     uint64_t n, uint32_t dims, uint32_t dtype,
                                                     uint32_t eb_mode, double eb,
                                                     DevParams* P) {
  __shared__ double red[7][kBlock];
  double v[7];
  for (int f = 0; f < 7; ++f) v[f] = f < 3 ? INFINITY : (f < 6 ? -INFINITY : 0.0);
  for (uint32_t b = threadIdx.x; b < nparts; b += blockDim.x)
    for (int f = 0; f < 7; ++f) {
      double u = partials[b * 8 + f];
      if (f < 3)
        v[f] = u < v[f] ? u : v[f];
      else
        v[f] = u > v[f] ? u : v[f];
    }
  for (int f = 0; f < 7; ++f) red[f][threadIdx.x] = v[f];
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int f = 0; f < 7; ++f)
    for (int t = 1; t < kBlock; ++t) {
      double u = red[f][t];
      if (f < 3)
        v[f] = u < v[f] ? u : v[f];
      else
        v[f] = u > v[f] ? u : v[f];
    }

  DevParams p;
  for (int d = 0; d < 3; ++d) p.lo[d] = p.hi[d] = 0.0, p.G[d] = 0;
  p.eb_user = eb;
  p.eb_abs = p.eb_eff = p.w = p.inv_w = 0.0;
  p.key16 = 1;
  p.status = BBX_OK;
  p.pad0 = 0;
  p.meta_bits = p.payload_bits = p.total_bytes = 0;
  for (int k = 0; k < 4; ++k) p.pad1[k] = 0;
  if (n == 0) {
    p.eb_abs = eb_mode == BBX_EB_ABS ? eb : 0.0;
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
    double rg = p.hi[d] - p.lo[d];
    if (rg > delta) delta = rg;
  }
  p.eb_abs = eb_mode == BBX_EB_REL ? eb * delta : eb;
  if (!isfinite(delta) || !isfinite(p.eb_abs)) {
    p.status = BBX_EBOUND;
    *P = p;
    return;
  }
  if (delta != 0.0) {
    double amax = 0.0;
    for (uint32_t d = 0; d < dims; ++d) {
      double a = fabs(p.lo[d]) > fabs(p.hi[d]) ? fabs(p.lo[d]) : fabs(p.hi[d]);
      if (a > amax) amax = a;
    }
    amax = amax + p.eb_abs;
    double guard = ldexp(amax, -48);
    if (dtype == BBX_F32) {
      int e = 0;
      (void)frexp(amax, &e);
      double half_ulp = ldexp(1.0, e - 25);
      double tiny = ldexp(1.0, -150);
      if (half_ulp < tiny) half_ulp = tiny;
      guard = guard + half_ulp;
    }
    p.eb_eff = p.eb_abs - guard;
    if (!(p.eb_eff > 0.0)) {
      p.status = BBX_EBOUND;
      *P = p;
      return;
    }
    p.w = 2.0 * p.eb_eff;
    p.inv_w = 1.0 / p.w;
    if (!isfinite(p.w) || !isfinite(p.inv_w) || !(p.inv_w > 0.0)) {
      p.status = BBX_EBOUND;
      *P = p;
      return;
    }
    for (uint32_t d = 0; d < dims; ++d) {
      double qm = floor((p.hi[d] - p.lo[d]) * p.inv_w + 0.5);
      if (!(qm < 1073741824.0)) {
        p.status = BBX_EBOUND;
        *P = p;
        return;
      }
      p.G[d] = bitlen32((uint32_t)qm);
      if (p.G[d] > 16) p.key16 = 0;
    }
  }
  *P = p;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_quantize(const T* pos, uint64_t n, uint32_t dims,
                                                     uint32_t layout, const DevParams* P,
                                                     void* keys, uint32_t* idx) {
  if (P->status != BBX_OK) return;
  const double inv_w = P->inv_w;
  const bool k16 = P->key16 != 0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    for (uint32_t d = 0; d < dims; ++d) {
      double x = load_coord(pos, n, dims, layout, i, d);
      uint32_t q = (uint32_t)floor((x - P->lo[d]) * inv_w + 0.5);
      if (k16)
        ((uint16_t*)keys)[(uint64_t)d * n + i] = (uint16_t)q;
      else
        ((uint32_t*)keys)[(uint64_t)d * n + i] = q;
    }
    if (idx) idx[i] = (uint32_t)i;
  }
}

hipError_t launch_range(const CompressPlan& p, const CompressWs& w, const void* pos,
                        hipStream_t s) {
  uint32_t nparts = 0;
  if (p.n > 0) {
    uint64_t want = (p.n + kBlock * 8 - 1) / (kBlock * 8);
    nparts = (uint32_t)(want < kMinMaxBlocks ? want : kMinMaxBlocks);
    if (p.dtype == BBX_F32)
      BBX_LAUNCH("range_minmax", k_minmax<float>, nparts, kBlock, 0, s, (const float*)pos, p.n,
                 p.dims, p.layout, w.partials);
    else
      BBX_LAUNCH("range_minmax", k_minmax<double>, nparts, kBlock, 0, s, (const double*)pos, p.n,
                 p.dims, p.layout, w.partials);
  }
  BBX_LAUNCH("range_epilogue", k_epilogue, 1, kBlock, 0, s, w.partials, nparts, p.n, p.dims,
             p.dtype, p.eb_mode, p.eb, w.params);
  if (p.n > 0) {
    uint64_t want = (p.n + kBlock * 4 - 1) / (kBlock * 4);
    uint32_t nb = (uint32_t)(want < 65536 ? want : 65536);
    uint32_t* idx = p.track_idx ? w.idx[0] : nullptr;
    if (p.dtype == BBX_F32)
      BBX_LAUNCH("quantize", k_quantize<float>, nb, kBlock, 0, s, (const float*)pos, p.n, p.dims,
                 p.layout, w.params, w.keys[0], idx);
    else
      BBX_LAUNCH("quantize", k_quantize<double>, nb, kBlock, 0, s, (const double*)pos, p.n,
                 p.dims, p.layout, w.params, w.keys[0], idx);
  }
  return hipGetLastError();
}

}  // namespace bbx

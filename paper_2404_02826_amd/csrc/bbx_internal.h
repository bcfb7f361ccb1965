// bbx_internal.h -- definitions shared by the HIP library's translation units.
// Not part of the public ABI (include/bitbox.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bitbox.h"

namespace bbx {

constexpr uint32_t kMagic = 0x31584242u;  // bytes 'B','B','X','1'
constexpr int kHeaderBytes = 128;
constexpr int kBlock = 256;               // threads per block for streaming kernels
constexpr int kMinMaxBlocks = 1024;       // partial-reduction blocks of the range pass
constexpr int kMaxDepth = 40;             // depth table size (n < 2^32 needs <= 33)
constexpr int kHistStride = 2048;         // per-node bins of the global radix select
constexpr int kRowStride = 258;           // per-chunk row: 257 prefix counts + below count

// Scalars of the range-and-bound step (Sec. 3), computed on the device by the
// range epilogue and read by every later compress kernel.
struct DevParams {
  double lo[3], hi[3];
  double eb_user, eb_abs, eb_eff, w, inv_w;
  uint32_t G[3];        // bits of the largest code per axis
  uint32_t key16;       // 1 when every code fits 16 bits
  uint32_t status;      // bbx_status of the call so far
  uint32_t pad0;
  uint64_t meta_bits, payload_bits, total_bytes;
  uint64_t pad1[4];
};

// Shape of the k-d tree, which depends on (n, r) only: at depth k every node
// holds a[k] = floor(n/2^k) or a[k]+1 particles (children of s are floor(s/2)
// and ceil(s/2)); L[k][t] counts the leaves under a node of a[k]+t particles.
struct TreeGeom {
  uint64_t n;
  uint32_t r;
  uint32_t depths;  // valid entries of a[] and L[]
  uint64_t a[kMaxDepth];
  uint64_t L[kMaxDepth][2];
};

TreeGeom make_geom(uint64_t n, uint32_t r);

// Per-leaf record used between the leaf, offset and packing kernels.
struct LeafRec {
  uint32_t start;    // first output slot
  uint32_t size;     // particles
  uint32_t m;        // widths m_x | m_y << 8 | m_z << 16
  uint32_t qref[3];  // codes of the reference particle
};

// Selection state of one node of a global level.
struct NodeSel {
  uint32_t prefix;  // high digits of the median code found so far
  uint32_t rank;    // rank of the median among the remaining candidates
  uint32_t v;       // median code (after the last pass)
  uint32_t jeq;     // members equal to v that go to the left child
};

// ---------------------------------------------------------------- device helpers

__host__ __device__ inline uint32_t bitlen32(uint32_t v) { return v ? 32u - (uint32_t)__builtin_clz(v) : 0u; }

// Node j of depth k: walk the path bits from the root (left child floor(s/2)).
__host__ __device__ inline void node_span(uint64_t n, uint32_t k, uint64_t j, uint64_t* start,
                                          uint64_t* size) {
  uint64_t s = n, st = 0;
  for (int b = (int)k - 1; b >= 0; --b) {
    uint64_t half = s >> 1;
    if ((j >> b) & 1u) {
      st += half;
      s -= half;
    } else {
      s = half;
    }
  }
  *start = st;
  *size = s;
}

__host__ __device__ inline uint64_t geom_L(const TreeGeom& g, uint32_t k, uint64_t s) {
  return g.L[k][s - g.a[k]];
}

// Leaf i (depth-first order): its first slot and size.
__host__ __device__ inline void leaf_span(const TreeGeom& g, uint64_t i, uint64_t* start,
                                          uint64_t* size) {
  uint64_t s = g.n, st = 0;
  uint32_t k = 0;
  while (s > g.r) {
    uint64_t sl = s >> 1;
    uint64_t Ll = geom_L(g, k + 1, sl);
    if (i < Ll) {
      s = sl;
    } else {
      i -= Ll;
      st += sl;
      s -= sl;
    }
    ++k;
  }
  *start = st;
  *size = s;
}

// Number of leaves before node j of depth k.
__host__ __device__ inline uint64_t leaves_before_node(const TreeGeom& g, uint32_t k, uint64_t j,
                                                       uint64_t start) {
  uint64_t big = start - j * g.a[k];  // nodes of a[k]+1 particles among the first j
  return j * g.L[k][0] + big * (g.L[k][1] - g.L[k][0]);
}

// Radix-select digit plan for a code of G bits: the last pass takes the low
// min(G, 8) bits; the bits above are split into one or two passes of <= 11.
struct DigitPlan {
  uint32_t npass;
  uint32_t width[3];
  uint32_t shift[3];
};

__host__ __device__ inline DigitPlan digit_plan(uint32_t G) {
  DigitPlan p;
  uint32_t wl = G < 8 ? G : 8;
  uint32_t rest = G - wl;
  if (rest == 0) {
    p.npass = 1;
    p.width[0] = wl;
  } else if (rest <= 11) {
    p.npass = 2;
    p.width[0] = rest;
    p.width[1] = wl;
  } else {
    p.npass = 3;
    p.width[0] = (rest + 1) / 2;
    p.width[1] = rest / 2;
    p.width[2] = wl;
  }
  uint32_t used = 0;
  for (uint32_t i = 0; i < p.npass; ++i) {
    used += p.width[i];
    p.shift[i] = G - used;
  }
  for (uint32_t i = p.npass; i < 3; ++i) p.width[i] = p.shift[i] = 0;
  return p;
}

// ---------------------------------------------------------------- launch plumbing

// Kernel timing hook (bbx_profile_*): records HIP events around a launch.
struct ProfScope {
  ProfScope(const char* name, hipStream_t s);
  ~ProfScope();
  const char* name;
  hipStream_t stream;
  hipEvent_t ev[2];
  bool on;
};

#define BBX_LAUNCH(name, kern, grid, block, shm, stream, ...)                  \
  do {                                                                          \
    ::bbx::ProfScope _bbx_ps(name, stream);                                     \
    hipLaunchKernelGGL(kern, dim3(grid), dim3(block), shm, stream, __VA_ARGS__); \
  } while (0)

// ---------------------------------------------------------------- launchers

struct CompressPlan {
  uint64_t n;
  uint32_t dims, dtype, layout, r, eb_mode, track_idx;
  double eb;
  uint32_t tile;          // tile capacity of the on-chip stage
  uint32_t global_levels; // depths handled by the global level kernels
  uint32_t tile_mode;     // 1: tile stage at depth global_levels, 0: big-leaf stage
  uint64_t n_leaves;
  uint64_t max_nodes;     // nodes of the deepest global level
  uint64_t max_blocks;    // blocks of the largest global level launch
  uint32_t mbits;
  TreeGeom geom;
};

struct CompressWs {
  DevParams* params;
  double* partials;
  void* keys[2];
  uint32_t* idx[2];
  uint32_t* hist;
  NodeSel* sel;
  uint32_t* rows;
  uint32_t* chunk_base;
  LeafRec* leaves;
  uint64_t* leaf_bits;
  uint64_t* scan_part;
};

struct LevelShape {
  uint32_t depth;
  uint64_t nodes;
  uint32_t iters;     // 256-element iterations per block
  uint64_t chunks;    // chunks per node
};

LevelShape level_shape(const CompressPlan& p, uint32_t depth);

hipError_t launch_range(const CompressPlan& p, const CompressWs& w, const void* pos,
                        hipStream_t s);
hipError_t launch_levels(const CompressPlan& p, const CompressWs& w, hipStream_t s, int* final_buf);
hipError_t launch_leaves(const CompressPlan& p, const CompressWs& w, int buf, uint32_t* perm,
                         hipStream_t s, int* out_buf);
hipError_t launch_scan(uint64_t count, uint64_t* bits, uint64_t* part, DevParams* params,
                       const CompressPlan* cp, uint64_t expect_payload, size_t out_cap,
                       uint64_t* d_size, hipStream_t s);
hipError_t launch_pack(const CompressPlan& p, const CompressWs& w, int buf, uint8_t* out,
                       uint64_t* d_size, uint32_t* d_status, hipStream_t s);

struct DecompressPlan {
  uint64_t n, n_leaves, meta_bits, payload_bits;
  uint32_t dims, dtype, r, mbits, layout;
  uint32_t G[3];
  double origin[3];
  double w;
  TreeGeom geom;
};

struct DecompressWs {
  DevParams* params;
  LeafRec* leaves;
  uint64_t* leaf_bits;
  uint64_t* scan_part;
};

hipError_t launch_decompress(const DecompressPlan& p, const DecompressWs& w, const uint8_t* stream,
                             void* pos, uint32_t* d_status, hipStream_t s);

uint64_t scan_blocks(uint64_t count);

}  // namespace bbx

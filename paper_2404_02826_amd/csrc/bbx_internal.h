// bbx_internal.h -- definitions shared by the HIP library's translation units.
// Not part of the public ABI (include/bitbox.h is).
//
// Every compress launch works on a batch of independent particle sets; a
// single compress is a batch of one.  Each kernel finds its set from the
// block index through a per-launch prefix array of block counts.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bitbox.h"

namespace bbx {

constexpr uint32_t kMagic = 0x31584242u;  // bytes 'B','B','X','1'
constexpr int kHeaderBytes = 128;
constexpr int kBlock = 256;               // threads per block for streaming kernels
constexpr int kMaxMinMaxBlocks = 1024;    // partial-reduction blocks of the range pass per set
constexpr int kMaxDepth = 40;             // depth table size (n < 2^32 needs <= 33)
constexpr int kHistBins = 256;            // per-node bins of the global radix select (digits <= 8 bits)
constexpr int kRowStride = 258;           // per-chunk row: 257 prefix counts + below count
constexpr int kRows = 8;                  // rows of kBlock elements per streaming group
constexpr int kGroup = kRows * kBlock;    // elements per streaming group
constexpr uint64_t kLevelBlocks = 4096;   // most blocks per global level (cap of a target or share)
constexpr uint64_t kSoloLevelBlocks = 1024;  // block target of a global level of a set alone
constexpr uint64_t kLocalBlocks = 4096;   // levels of at least this many nodes run block-local
constexpr uint32_t kStageChunk = 16384;   // the global scatter stages groups from this chunk size
constexpr uint32_t kRedLdsBoxes = 4096;
// Status of a set whose bound the grid cannot meet (eb_eff <= 0 or codes of
// 30 bits or more): every later kernel skips it as it skips a failed set,
// the packer stores its coordinates as they are (Sec. 4.1's lossless
// escape), and it is reported as BBX_OK.
constexpr uint32_t kStatusLossless = 0x100;   // bit box reduction: boxes kept in LDS (24 B each)
// a block-local level is one chunk per node under every block target
static_assert(kLevelBlocks <= kLocalBlocks, "block-local levels must have one chunk per node");

// Scalars of the range-and-bound step (Sec. 3), computed on the device by the
// range epilogue and read by every later compress kernel of the set.
struct DevParams {
  double lo[3], hi[3];
  double eb_user, eb_abs, eb_eff, w, inv_w;
  uint32_t G[3];        // bits of the largest code per axis
  uint32_t key16;       // 1 when every code fits 16 bits
  uint32_t status;      // bbx_status of the set so far
  uint32_t diag;        // first internal consistency check that failed (Check), 0 if none
  uint64_t meta_bits, payload_bits, total_bytes;
  uint64_t payload_base;  // global payload-bit offset of the set's first leaf
  uint64_t nseq;          // sequences of the version-2 stream (reduce or split-rule sets)
  uint64_t nleaves;       // leaves the partition made (split-rule sets; found on the device)
  uint64_t pad1[1];
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
  uint32_t ref_src;  // source index of the reference (compress, when indices are carried)
};

// Selection state of one node of a global level.
struct NodeSel {
  uint32_t prefix;  // high digits of the median code found so far
  uint32_t rank;    // rank of the median among the remaining candidates
  uint32_t v;       // median code (after the last pass)
  uint32_t jeq;     // members equal to v that go to the left child
};

// One set of a compress batch (device-resident).
struct SetDesc {
  const void* pos;        // caller's positions
  uint8_t* out;           // caller's stream buffer
  uint32_t* perm;         // optional source index per output slot
  uint64_t* d_size;       // optional stream length (UINT64_MAX on error)
  uint32_t* d_status;     // optional status
  uint64_t n, out_cap;
  uint64_t kst;           // element stride between the code arrays of two axes (n rounded up to 64)
  double eb;
  uint32_t dims, dtype, layout, r, eb_mode, mbits;
  uint32_t gl;            // global levels
  uint32_t tile_mode;     // 1: tile stage at depth gl; 0: big-leaf stage
  uint32_t final_buf;     // key buffer that ends in output-slot order
  uint32_t mm_blocks;     // blocks of the range pass
  uint32_t level_blocks;  // block target of the set's global levels (level_shape)
  uint32_t ref_rule;      // leaf reference: 0 nearest the AABB centre, 1 fewest code bits
  uint32_t ref_mode;      // reference stored as 0 its codes, 1 its original coordinates
  uint32_t track;         // source indices follow the codes (perm output or ref_mode 1)
  uint32_t fuse_depth;    // depth k whose levels k, k + 1 run fused in place, a wavefront per node (kNoFuse: none)
  uint32_t fuse_depth4;   // the same with a block per node (nodes of at most 4 kFuseNode)
  uint32_t reduce;        // bit box reduction: 0 none, 1 key sum of widths, 2 key sum of lengths
  uint32_t* user_perm;    // the caller's perm output of a reduce or split-rule set (perm then points into the workspace)
  uint32_t split;         // split rule: 0 the median partition above; 1-3 the ablations (k_split.hip)
  uint32_t sp_levels;     // split-rule sets: global split levels launched
  uint64_t sp_off;        // split-rule sets: byte offset of the set's region in Ws::split
  uint64_t n_leaves;
  uint64_t key_off;       // byte offset into each key buffer (capacity dims*n*4)
  uint64_t idx_off;       // u32 offset into each index buffer
  uint64_t hist_off;      // u32 offset into the histogram bins
  uint64_t hist_half;     // u32 entries of each of the set's two bin regions
  uint64_t sel_off;       // NodeSel offset
  uint64_t sel_half;      // NodeSel entries of each of the set's two selection regions (by depth parity)
  uint64_t rows_off;      // u32 offset into the chunk rows
  uint64_t cb_off;        // u32 offset into the chunk bases
  uint64_t cb_half;       // u32 entries of each of the set's two chunk-base regions (by depth parity)
  uint64_t lab_off;       // u64 offset into the side labels of paired levels
  uint32_t npairs;        // global levels 2p and 2p + 1 (p < npairs) run with one data movement
  uint32_t fuse_depth16;  // the pair of fuse_depth4 with a block of 16 wavefronts per node (at most 16 kFuseNode)
  uint64_t leaf_off;      // first leaf of the set in the batch's leaf arrays
  uint64_t part_off;      // first block of the set's range partials
  TreeGeom geom;
};

// Shared scratch of a batch.
struct Ws {
  DevParams* params;   // [nsets]
  const SetDesc* sets; // [nsets]
  double* partials;    // range partials, 8 doubles per block
  uint8_t* keys[2];
  uint32_t* idx[2];
  uint32_t* hist;
  NodeSel* sel;
  uint32_t* rows;
  uint32_t* chunk_base;
  uint64_t* labels;     // side labels of a paired level's members, one bit each
  LeafRec* leaves;
  uint64_t* leaf_bits;
  uint64_t* scan_part;
  uint64_t* scan_total;
  const uint64_t* pre;  // block-count prefix arrays (see BatchPlan)
  uint32_t* pass_need;  // [kMaxDepth][4]: some set runs mid pass p at depth k
  uint32_t* tile_defer; // [0] = count, then global tile indices left to the 32-bit tile pass
  uint32_t* lossless;   // [0] = count, then the sets stored losslessly
  // bit box reduction (sets with reduce != 0), particle arrays at idx_off, leaf arrays at leaf_off
  uint4* red_tq;
  uint8_t* red_taken;
  uint32_t* red_slot;
  uint64_t* red_key;
  uint4* red_ctr;
  uint32_t* red_ref;
  uint32_t* red_hits;
  uint4* red_seq;
  uint8_t* split;       // partition state of the split-rule sets (SpLayout per set)
};

// A set's stream holds one record per sequence (version 2): the bit box
// reduction, or a split rule other than 0 (one sequence per leaf).
__host__ __device__ inline bool seq_stream(const SetDesc& S) { return S.reduce != 0 || S.split != 0; }

// Paired global levels: depths 2p and 2p + 1 (p < npairs) partition the
// codes with one data movement (k_pair.hip), so the key buffer that holds a
// level's codes is the depth minus the pairs before it, mod 2.
__host__ __device__ inline bool pair_first(const SetDesc& S, uint32_t depth) {
  return (depth & 1u) == 0 && depth / 2 < S.npairs;
}
__host__ __device__ inline bool pair_second(const SetDesc& S, uint32_t depth) {
  return (depth & 1u) && depth / 2 < S.npairs;
}
__host__ __device__ inline uint32_t key_buf(const SetDesc& S, uint32_t depth) {
  return (depth - (depth / 2 < S.npairs ? depth / 2 : S.npairs)) & 1u;
}
// the node selections and chunk bases of a global level: two regions by
// depth parity (a paired level reads its first level's while it writes its
// second's)
__host__ __device__ inline NodeSel* sel_level(const SetDesc& S, uint32_t depth, NodeSel* sel0) {
  return sel0 + S.sel_off + (depth & 1u) * S.sel_half;
}
__host__ __device__ inline const NodeSel* sel_level(const SetDesc& S, uint32_t depth, const NodeSel* sel0) {
  return sel0 + S.sel_off + (depth & 1u) * S.sel_half;
}
__host__ __device__ inline uint32_t* cb_level(const SetDesc& S, uint32_t depth, uint32_t* cb0) {
  return cb0 + S.cb_off + (depth & 1u) * S.cb_half;
}
__host__ __device__ inline const uint32_t* cb_level(const SetDesc& S, uint32_t depth, const uint32_t* cb0) {
  return cb0 + S.cb_off + (depth & 1u) * S.cb_half;
}

// widths of a box packed m_x | m_y << 8 | m_z << 16
__device__ inline uint32_t red_m(uint32_t mp, uint32_t d) { return (mp >> (8 * d)) & 0xffu; }

// Reduction key of a box: (sum of widths, or with reduce = 2 the sum of
// Eq. 3 box lengths in units of 2 eps) << 31 | leaf (leaf < 2^31), the order
// of (key, leaf).
__device__ inline uint64_t red_key(uint32_t mp, uint32_t dims, uint32_t rule, uint32_t leaf) {
  uint64_t k = 0;
  for (uint32_t d = 0; d < dims; ++d) {
    const uint32_t m = red_m(mp, d);
    k += rule == 2 ? ((1ull << m) - 1) : m;
  }
  return (k << 31) | leaf;
}

// Eq. 2 width of a largest offset D: bitlen(D) + 1, zero when D = 0.
__device__ inline uint32_t red_width(uint32_t D) { return D ? 33u - (uint32_t)__builtin_clz(D) : 0u; }

// ---------------------------------------------------------------- split rules 1-3

constexpr uint32_t kSpTile = 2048;   // particles per tile of a global split level (256 threads x 8)
constexpr uint32_t kSpLocal = 1024;  // nodes of at most this many particles finish in one block

// A node of the split-rule partition (32 bytes): its particles are
// positions [start, start + size) of the set's tree order.  Rule 2: the
// leaves [i0, i1) it will hold.  Rule 3: its cell, codes lo[d] ..
// lo[d] + 2^lg[d] - 1.  pk = lg[0] | lg[1] << 5 | lg[2] << 10 | buf << 16 |
// leaf << 17 | depth << 24 (buf: which element buffer holds the particles).
struct SpNode {
  uint32_t start, size, i0, i1;
  uint32_t lo[3];
  uint32_t pk;
};
__host__ __device__ inline uint32_t sp_lg(uint32_t pk, uint32_t d) { return (pk >> (5 * d)) & 31u; }
__host__ __device__ inline uint32_t sp_depth(uint32_t pk) { return pk >> 24; }

// Per active node of a global split level: the split and the selection state.
struct SpSel {
  uint32_t axis, npass, prefix, rank;  // radix selection of the rank-k code (rules 1, 2)
  uint32_t k;                          // rank of the split (rules 1, 2), midpoint code (rule 3)
  uint32_t nl;                         // left child size
  uint32_t tile0;                      // first tile of the node in the level's tile list
  uint32_t base_lt, base_eq;           // the level-wide tile scan at the node's first tile
  uint32_t ext[6];                     // rule 1: code min, max per axis
  uint32_t pad;
};

// Control words of a set's split partition.
enum { kSpNa0 = 0, kSpNa1 = 1, kSpTiles = 2, kSpDone = 3, kSpCovered = 4, kSpCtlWords = 16 };

// Byte offsets inside one set's split region.  na: active nodes of a level
// (each holds more than kSpLocal particles, disjoint); ta: tiles of a level;
// dc: done nodes (children that are leaves or fit one block; disjoint and
// non-empty, at most two per active node of each level).
struct SpLayout {
  uint64_t na, ta, dc, np;
  uint64_t e[2], len, nodes[2], sel, hist, tcnt, toff, done, part, ctl, total;
};
__host__ __device__ inline SpLayout sp_layout(uint64_t n, uint32_t levels) {
  SpLayout L;
  L.na = n / (kSpLocal + 1) + 1;
  L.ta = (n + kSpTile - 1) / kSpTile + L.na;
  const uint64_t dc = 2 * (uint64_t)levels * L.na + 1;
  L.dc = dc < n + 1 ? dc : n + 1;
  L.np = (n + kSpTile - 1) / kSpTile + 1;
  uint64_t off = 0;
  auto take = [&](uint64_t bytes) {
    const uint64_t o = off;
    off = (off + bytes + 255) & ~(uint64_t)255;
    return o;
  };
  L.e[0] = take(16 * n);
  L.e[1] = take(16 * n);
  L.len = take(4 * n);
  L.nodes[0] = take(sizeof(SpNode) * L.na);
  L.nodes[1] = take(sizeof(SpNode) * L.na);
  L.sel = take(sizeof(SpSel) * L.na);
  L.hist = take(4 * 256 * L.na);
  L.tcnt = take(8 * L.ta);
  L.toff = take(8 * L.ta);
  L.done = take(sizeof(SpNode) * L.dc);
  L.part = take(4 * L.np);
  L.ctl = take(4 * kSpCtlWords);
  L.total = off;
  return L;
}

// ---------------------------------------------------------------- device helpers

// Internal consistency checks of the partition and leaf kernels.  None can
// fail on a correct build; a failing one sets the set's status to BBX_EHIP
// and records which check failed first (DevParams::diag), which the host
// reports in bbx_last_error.
enum Check : uint32_t {
  kChkLastDigit = 1,    // a node's last-digit bins hold fewer members than the median's rank
  kChkLastDigitWide = 2,
  kChkScatterStore = 3, // a member's slot falls outside its node
  kChkScatterStage = 4, // a member's staged slot falls outside its group
  kChkScatterDrain = 5,
  kChkStageIdx = 6,     // staged partition without carried indices
  kChkWavePart = 7,
  kChkFusedIdx = 8,
  kChkFusedPart = 9,
  kChkTileLeaves = 10,  // leaf count of a tile differs from the tree geometry
  kChkTileRange = 11,
  kChkReduce = 12,      // the reduction did not place every particle
  kChkSplit = 13,       // a split-rule partition overflowed its node lists or left particles out
  kChkPairStage = 14,   // a paired level's member falls outside its group's staging
  kChkPairStore = 15,   // a paired level's member falls outside its node
};
__device__ inline void check_failed(DevParams* P, uint32_t which) {
  atomicCAS(&P->diag, 0u, which);
  P->status = BBX_EHIP;
}

__host__ __device__ inline uint32_t bitlen32(uint32_t v) { return v ? 32u - (uint32_t)__builtin_clz(v) : 0u; }

// Bits of one stored original coordinate (M of Sec. 4.2): 32 for f32, 64 for f64.
__host__ __device__ inline uint32_t coord_bits(uint32_t dtype) { return dtype == BBX_F32 ? 32u : 64u; }

// Node j of depth k: walk the path bits from the root (left child floor(s/2)).
__host__ __device__ inline void node_span(uint64_t n, uint32_t k, uint64_t j, uint64_t* start,
                                          uint64_t* size) {
  if ((n & ((1ull << k) - 1)) == 0) {  // 2^k divides n: every node of depth k holds n / 2^k
    *size = n >> k;
    *start = j * (n >> k);
    return;
  }
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
// min(G, 8) bits; the bits above are split evenly into passes of <= 8 bits.
struct DigitPlan {
  uint32_t npass;
  uint32_t width[4];
  uint32_t shift[4];
};

__host__ __device__ inline DigitPlan digit_plan(uint32_t G) {
  DigitPlan p;
  const uint32_t wl = G < 8 ? G : 8;
  const uint32_t rest = G - wl;
  const uint32_t nmid = (rest + 7) / 8;  // 0..3 for G <= 30
  p.npass = nmid + 1;
  const uint32_t base = nmid ? rest / nmid : 0, extra = nmid ? rest % nmid : 0;
  // mid passes (the first `extra` get one more bit), then the last digit
  p.width[0] = nmid >= 1 ? base + (extra > 0 ? 1u : 0u) : wl;
  p.width[1] = nmid >= 2 ? base + (extra > 1 ? 1u : 0u) : (nmid == 1 ? wl : 0u);
  p.width[2] = nmid >= 3 ? base : (nmid == 2 ? wl : 0u);
  p.width[3] = nmid == 3 ? wl : 0u;
  p.shift[0] = G - p.width[0];
  p.shift[1] = p.shift[0] - p.width[1];
  p.shift[2] = p.shift[1] - p.width[2];
  p.shift[3] = p.shift[2] - p.width[3];
  return p;
}

// width / shift of pass i without dynamic indexing (keeps the plan in registers)
__host__ __device__ inline uint32_t dp_width(const DigitPlan& p, uint32_t i) {
  return i == 0 ? p.width[0] : (i == 1 ? p.width[1] : (i == 2 ? p.width[2] : p.width[3]));
}
__host__ __device__ inline uint32_t dp_shift(const DigitPlan& p, uint32_t i) {
  return i == 0 ? p.shift[0] : (i == 1 ? p.shift[1] : (i == 2 ? p.shift[2] : p.shift[3]));
}

// Blocks of one global level of one set: nodes x chunks, each chunk a whole
// number of streaming groups, about target_blocks blocks per level.  A set
// alone targets kSoloLevelBlocks; in a batch each set targets its share of
// 4 kLevelBlocks (by particle count, at least 1), so that a batch of many small sets does
// not launch a block per 2048 codes.  Which levels are global does not depend
// on the target (level_kind below asks for kLocalBlocks).
struct LevelShape {
  uint64_t nodes;
  uint32_t chunk_elems;
  uint64_t chunks;
};

__host__ __device__ inline LevelShape level_shape(uint64_t n, uint32_t depth,
                                                  uint64_t target_blocks) {
  LevelShape sh;
  sh.nodes = 1ull << depth;
  const uint64_t maxsz = (n + sh.nodes - 1) >> depth;  // ceil(n / 2^depth)
  uint64_t cpn = (target_blocks + sh.nodes - 1) / sh.nodes;
  if (cpn == 0) cpn = 1;
  const uint64_t elems = (maxsz + cpn - 1) / cpn;
  uint64_t groups = (elems + kGroup - 1) / kGroup;
  if (groups < 1) groups = 1;
  sh.chunk_elems = (uint32_t)(groups * kGroup);
  sh.chunks = (maxsz + sh.chunk_elems - 1) / sh.chunk_elems;
  if (sh.chunks == 0) sh.chunks = 1;
  return sh;
}

// How a global level of a set runs.  Nodes of at most kWaveNode members: one
// wavefront per node (k_level_wave).  Otherwise, nodes that each fit one
// block (one chunk per node): one block per node (k_level_local).  Both find
// the median and partition the node with no global histograms or chunk
// tables.  Otherwise: global histograms over chunks.  Node sizes only shrink
// with depth, so the global levels come first.
constexpr uint64_t kWaveNode = 4096;
enum { kLevelGlobal = 0, kLevelBlock = 1, kLevelWave = 2 };
__host__ __device__ inline int level_kind(uint64_t n, uint32_t depth) {
  if (((n + (1ull << depth) - 1) >> depth) <= kWaveNode) return kLevelWave;
  return level_shape(n, depth, kLocalBlocks).chunks == 1 ? kLevelBlock : kLevelGlobal;
}
__host__ __device__ inline bool level_is_local(uint64_t n, uint32_t depth) {
  return level_kind(n, depth) != kLevelGlobal;
}

// Radix bins of a level's nodes (256 per node): global levels use the set's
// first region; a block-local level of depth k uses region k & 1, since its
// kernel reads its own nodes' first-digit bins while it builds those of the
// next level's nodes.
__device__ inline uint32_t* hist_level(const SetDesc& S, uint32_t depth, uint32_t* hist) {
  return level_kind(S.n, depth) == kLevelBlock ? hist + (depth & 1) * S.hist_half : hist;
}

// The last levels above the tile stage of a set with a tile stage run in
// in-place pairs with the node in registers: depths gl - 2 and gl - 1 when
// their nodes have at most kFuseNode members (a wavefront per node), depths
// gl - 4 and gl - 3 when theirs have at most 4 kFuseNode (a block of four
// wavefronts per node), and depths gl - 6 and gl - 5 when theirs have at
// most 16 kFuseNode and there are at least kFuse16Nodes of them (a block of
// 16 wavefronts per node, one per CU: it pays off over the levels of large
// sets, not over the few ragged nodes of small ones).
// Each pair leaves the data of depth k + 2 in the buffer of depth k, which
// has its parity.
constexpr uint64_t kFuseNode = 1024;
constexpr uint32_t kNoFuse = 0x80000000u;  // depth - kNoFuse >= 2 for every depth (unsigned)
constexpr uint64_t kFuse16Nodes = 1024;     // fewest nodes of a 16-wavefront pair's first level
__host__ __device__ inline uint32_t fuse_depth_of(uint64_t n, uint32_t gl, bool tile_mode,
                                                  uint32_t back, uint64_t max_node) {
  if (!tile_mode || gl < back) return kNoFuse;
  const uint32_t k = gl - back;
  return ((n + (1ull << k) - 1) >> k) <= max_node ? k : kNoFuse;
}
// depth is a level of one of the set's fused pairs
__host__ __device__ inline bool level_fused(const SetDesc& S, uint32_t depth) {
  return depth - S.fuse_depth < 2u || depth - S.fuse_depth4 < 2u || depth - S.fuse_depth16 < 2u;
}

// Leaves per block of the leaf-aligned packing and unpacking kernels: at most
// 2048 slots and 256 leaves per block.
__host__ __device__ inline uint32_t leaves_per_block(uint32_t r) {
  const uint32_t l = r >= 2048 ? 1u : 2048u / r;
  return l < 256u ? l : 256u;
}

// set owning global block b: largest s with pre[s] <= b (pre non-decreasing,
// pre[0] = 0, b < pre[nsets])
__device__ inline uint32_t find_set(const uint64_t* pre, uint32_t nsets, uint64_t b) {
  uint32_t lo = 0, hi = nsets - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// ---------------------------------------------------------------- wavefront helpers

// Inclusive scan over the 64 lanes with DPP row shifts and row broadcasts (no
// LDS traffic): rows of 16 lanes first, then row 0's total into row 1, row
// 2's into row 3, and rows 0-1's total into rows 2-3.  Lanes whose source is
// outside the row read 0.
__device__ inline uint32_t wave_incl(uint32_t x) {
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);  // row_shr:1
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);  // row_shr:2
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);  // row_shr:4
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);  // row_shr:8
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);  // row_bcast:15
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return x;
}

// Orders the wavefront's LDS accesses around a phase boundary (no cross-wave
// synchronization is needed: each wavefront owns its tile).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline uint32_t umin32(uint32_t a, uint32_t b) { return a < b ? a : b; }
__device__ inline uint32_t umax32(uint32_t a, uint32_t b) { return a > b ? a : b; }
// wavefront minimum / maximum, uniform result
__device__ inline uint32_t wave_min_dpp(uint32_t x) {
  const int I = -1;  // identity of min (0xffffffff)
  x = umin32(x, (uint32_t)__builtin_amdgcn_update_dpp(I, (int)x, 0x111, 0xf, 0xf, false));
  x = umin32(x, (uint32_t)__builtin_amdgcn_update_dpp(I, (int)x, 0x112, 0xf, 0xf, false));
  x = umin32(x, (uint32_t)__builtin_amdgcn_update_dpp(I, (int)x, 0x114, 0xf, 0xf, false));
  x = umin32(x, (uint32_t)__builtin_amdgcn_update_dpp(I, (int)x, 0x118, 0xf, 0xf, false));
  x = umin32(x, (uint32_t)__builtin_amdgcn_update_dpp(I, (int)x, 0x142, 0xa, 0xf, false));
  x = umin32(x, (uint32_t)__builtin_amdgcn_update_dpp(I, (int)x, 0x143, 0xc, 0xf, false));
  return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}
__device__ inline uint32_t wave_max_dpp(uint32_t x) {
  x = umax32(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false));
  x = umax32(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false));
  x = umax32(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false));
  x = umax32(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false));
  x = umax32(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false));
  x = umax32(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false));
  return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}

// set bits of a wavefront mask in the lanes below this one
__device__ inline uint32_t lanes_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
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

// Host-side launch plan of a batch: grid sizes and the offsets (in u64
// entries) of each prefix array inside the uploaded plan buffer.
// kernel families of a set's global level (which launch handles it)
constexpr uint8_t kFamNone = 0;    // second level of a fused pair
constexpr uint8_t kFamGlobal = 1;  // global histograms, single or paired
constexpr uint8_t kFamLocal = 2;   // a block per node
constexpr uint8_t kFamWave = 3;    // a wavefront per node
constexpr uint8_t kFamFused = 4;   // two levels, a wavefront per node
constexpr uint8_t kFamFused4 = 5;  // two levels, a block per node
constexpr uint8_t kFamFused16 = 6; // two levels, a block of 16 wavefronts per node

struct BatchPlan {
  uint32_t nsets;
  uint32_t max_gl;            // deepest global level count over the sets
  uint32_t tile;              // tile capacity (256 or 512)
  uint32_t track;             // source indices are carried (some set wants perm or ref_mode 1)
  uint64_t total_leaves;
  uint64_t hist_entries;      // u32 bins zeroed once per call
  uint64_t g_mm, g_qz, g_tile, g_big, g_pm, g_pp;
  uint64_t o_mm, o_qz, o_tile, o_big, o_pm, o_pp;
  // per depth: global levels' chunk blocks and nodes, block-local levels'
  // blocks, wavefront levels' nodes, fused pairs' nodes (a wavefront or a
  // block each); each array counts only the sets of its family at that depth
  uint64_t g_lv[kMaxDepth], g_nd[kMaxDepth], g_lc[kMaxDepth], g_wv[kMaxDepth];
  uint64_t g_fu[kMaxDepth], g_f4[kMaxDepth], g_f16[kMaxDepth];
  uint64_t o_lv[kMaxDepth], o_nd[kMaxDepth], o_lc[kMaxDepth], o_wv[kMaxDepth];
  uint64_t o_fu[kMaxDepth], o_f4[kMaxDepth], o_f16[kMaxDepth];
  uint8_t lv_local[kMaxDepth];   // some set handles level k one block per node
  uint8_t lv_global[kMaxDepth];  // some set handles level k with global histograms
  uint8_t sel_wide[kMaxDepth];   // some set's nodes have > 256 chunks at global level k
  uint8_t scat_stage[kMaxDepth]; // every set's chunks at global level k hold >= kStageChunk codes
  uint8_t lv_wave[kMaxDepth];    // some set handles level k one wavefront per node
  uint8_t lv_fused[kMaxDepth];   // some set handles levels k, k + 1 fused, a wavefront per node
  uint8_t lv_fused4[kMaxDepth];  // some set handles levels k, k + 1 fused, a block per node
  uint8_t lv_fused16[kMaxDepth]; // the same with a block of 16 wavefronts per node
  uint8_t lv_single[kMaxDepth];  // some set partitions global level k alone (k_scatter)
  uint8_t lv_pair[kMaxDepth];    // some set partitions global levels k, k + 1 together (k_pair.hip)
  uint8_t pair_wide[kMaxDepth];  // some paired set's nodes have > 256 chunks at level k
  uint32_t reduce;               // some set runs the bit box reduction
  uint32_t red_lds_boxes;        // some reduce set keeps its boxes on chip (<= kRedLdsBoxes leaves)
  uint32_t red_global;           // some reduce set keeps them in the workspace
  uint32_t split;                // some set uses a split rule other than 0
  uint64_t g_rp, g_rl, g_rw;     // reduction: preparation, loop and packing blocks
  uint64_t o_rp, o_rl, o_rw;
  uint64_t pre_entries;       // total u64 entries of the prefix buffer
};

// The 128 header bytes the host planned a decode from; the decoder's first
// kernel compares them with the stream's own header (a mismatch makes the
// stream corrupt).
struct HeaderCopy {
  uint64_t w[kHeaderBytes / 8];
};

struct DecompressPlan {
  HeaderCopy header;
  uint32_t version;  // 1: one record per leaf; 2: one per sequence of the bit box reduction
  uint64_t n_seq;
  uint64_t n, n_leaves, meta_bits, payload_bits;
  uint32_t dims, dtype, r, mbits, layout, ref_mode;
  uint32_t G[3];
  double origin[3];
  double w, inv_w;
  TreeGeom geom;
};

struct DecompressWs {
  DevParams* params;
  LeafRec* leaves;
  uint64_t* leaf_bits;
  uint64_t* scan_part;
  uint64_t* slot_start;  // version 2: first output slot of each sequence
};

uint64_t scan_blocks(uint64_t count);

// Sets the calling thread's error message (bbx_last_error) and returns st.
bbx_status set_error(bbx_status st, const char* msg);

// launchers (one group per translation unit)
hipError_t launch_range(const BatchPlan& bp, const Ws& w, hipStream_t s);
hipError_t launch_levels(const BatchPlan& bp, const Ws& w, hipStream_t s);
hipError_t launch_pair(const BatchPlan& bp, const Ws& w, uint32_t depth, hipStream_t s);
hipError_t launch_leaves(const BatchPlan& bp, const Ws& w, hipStream_t s);
hipError_t launch_pack(const BatchPlan& bp, const Ws& w, hipStream_t s);
hipError_t launch_decompress(const DecompressPlan& p, const DecompressWs& w, const uint8_t* stream,
                             void* pos, uint32_t* d_status, hipStream_t s);
hipError_t launch_export(const DecompressPlan& p, const DecompressWs& w, const uint8_t* stream,
                         void* out, uint32_t* d_status, hipStream_t s);
hipError_t launch_dec_scan(uint64_t count, uint64_t* bits, uint64_t* part, DevParams* params,
                           uint64_t expect_payload, hipStream_t s);
hipError_t launch_reduce(const BatchPlan& bp, const Ws& w, hipStream_t s);
hipError_t launch_split(const BatchPlan& bp, const SetDesc* descs, const Ws& w, hipStream_t s);
hipError_t launch_reorder_hist(uint64_t n_leaves, uint32_t dims, const DecompressWs& w,
                               uint32_t* whist, uint8_t* key, uint32_t* bcount, hipStream_t s);
hipError_t launch_reorder_write(const DecompressPlan& p, const DecompressWs& w, const uint32_t ord[3],
                                const uint8_t* plain, uint8_t* out, uint64_t out_words, uint8_t* key,
                                uint32_t* bcount, uint32_t* order, uint64_t* sbits, hipStream_t s);
hipError_t launch_reduce_pack(const BatchPlan& bp, const Ws& w, hipStream_t s);
hipError_t launch_decompress2(const DecompressPlan& p, const DecompressWs& w, const uint8_t* stream,
                              void* pos, hipStream_t s);

}  // namespace bbx

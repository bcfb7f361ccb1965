// abi.hip -- the C ABI of include/bitbox.h: argument validation, the launch
// plan (tree shape, tile depth), workspace carving, the stream-ordered launch
// sequence, and kernel timing.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "bbx_internal.h"

namespace bbx {

static thread_local std::string g_err;

static bbx_status fail(bbx_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

bbx_status set_error(bbx_status st, const char* msg) { return fail(st, msg); }

// ---------------------------------------------------------------- profiling

struct ProfEntry {
  std::string name;
  uint64_t launches = 0;
  double ms = 0.0;
};
struct Pending {
  int entry;
  hipEvent_t ev[2];
};
static std::mutex g_prof_mu;
static bool g_prof_on = false;
static std::vector<ProfEntry> g_prof;
static std::vector<Pending> g_pending;

static int prof_index(const char* name) {
  for (size_t i = 0; i < g_prof.size(); ++i)
    if (g_prof[i].name == name) return (int)i;
  ProfEntry e;
  e.name = name;
  g_prof.push_back(e);
  return (int)g_prof.size() - 1;
}

ProfScope::ProfScope(const char* nm, hipStream_t s) : name(nm), stream(s), on(false) {
  if (!g_prof_on) return;
  if (hipEventCreate(&ev[0]) != hipSuccess) return;
  if (hipEventCreate(&ev[1]) != hipSuccess) {
    (void)hipEventDestroy(ev[0]);
    return;
  }
  (void)hipEventRecord(ev[0], stream);
  on = true;
}

ProfScope::~ProfScope() {
  if (!on) return;
  (void)hipEventRecord(ev[1], stream);
  std::lock_guard<std::mutex> lk(g_prof_mu);
  Pending p;
  p.entry = prof_index(name);
  p.ev[0] = ev[0];
  p.ev[1] = ev[1];
  g_pending.push_back(p);
}

static void prof_drain() {
  for (auto& p : g_pending) {
    float ms = 0.f;
    if (hipEventSynchronize(p.ev[1]) == hipSuccess &&
        hipEventElapsedTime(&ms, p.ev[0], p.ev[1]) == hipSuccess) {
      g_prof[p.entry].launches += 1;
      g_prof[p.entry].ms += ms;
    }
    (void)hipEventDestroy(p.ev[0]);
    (void)hipEventDestroy(p.ev[1]);
  }
  g_pending.clear();
}

// ---------------------------------------------------------------- geometry

TreeGeom make_geom(uint64_t n, uint32_t r) {
  TreeGeom g;
  memset(&g, 0, sizeof(g));
  g.n = n;
  g.r = r;
  uint32_t D = 0;
  while (D < 63 && ((n + (1ull << D) - 1) >> D) > r) ++D;  // first depth with every node <= r
  g.depths = D + 1;
  for (uint32_t k = 0; k <= D && k < (uint32_t)kMaxDepth; ++k) g.a[k] = n >> k;
  for (int k = (int)D; k >= 0; --k)
    for (int t = 0; t < 2; ++t) {
      uint64_t s = g.a[k] + t;
      if (s <= r || k == (int)D) {
        g.L[k][t] = 1;
      } else {
        uint64_t sl = s >> 1, sr = s - sl;
        g.L[k][t] = g.L[k + 1][sl - g.a[k + 1]] + g.L[k + 1][sr - g.a[k + 1]];
      }
    }
  return g;
}

static size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

// Leaves of a split-rule partition at most: rule 1 those of the halving
// recursion, rule 2 ceil(n / r), rule 3 one per particle.
static uint64_t split_leaf_cap(uint64_t n, uint32_t r, uint32_t rule) {
  if (n == 0) return 0;
  if (rule == 2) return (n + r - 1) / r;
  if (rule == 3) return n;
  return make_geom(n, r).L[0][0];
}

// Global levels a split-rule partition launches: until every node is a leaf
// or holds at most kSpLocal particles (rule 1: nodes of depth k hold at most
// ceil(n / 2^k); rule 2: at most ceil(b / 2^k) leaves of at most ceil(n / b)
// particles; rule 3: every halving narrows one axis of a cell of at most 30
// bits, so 30 dims levels leave single codes).
static uint32_t split_levels(uint64_t n, uint32_t r, uint32_t rule, uint32_t dims) {
  if (rule == 3) return 30 * dims;
  uint32_t k = 0;
  if (rule == 2) {
    const uint64_t b = (n + r - 1) / r, lsz = b ? (n + b - 1) / b : 0;
    while (true) {
      const uint64_t lv = (b + (1ull << k) - 1) >> k;
      if (lv <= 1 || lv * lsz <= kSpLocal) return k;
      ++k;
    }
  }
  const uint64_t cap = std::max<uint64_t>(kSpLocal, r);
  while (((n + (1ull << k) - 1) >> k) > cap) ++k;
  return k;
}

// One set of a compress request, as the ABI receives it.
struct SetIn {
  const void* pos;
  uint64_t n;
  uint32_t dims;
  bbx_dtype dtype;
  double eb;
  bbx_params prm;
  void* out;
  size_t out_cap;
  uint64_t* d_size;
  uint32_t* d_status;
  uint32_t* d_perm;
  bool need_idx;  // plan source-index buffers (a perm output or ref_mode 1)
};

static bbx_status check_compress_args(uint64_t n, uint32_t dims, bbx_dtype dtype, double eb,
                                      const bbx_params* prm) {
  if (!prm) return fail(BBX_EINVAL, "params is NULL");
  if (dtype != BBX_F32 && dtype != BBX_F64) return fail(BBX_EINVAL, "dtype must be BBX_F32 or BBX_F64");
  if (prm->layout != BBX_AOS && prm->layout != BBX_SOA) return fail(BBX_EINVAL, "layout must be AOS or SOA");
  if (prm->eb_mode != BBX_EB_REL && prm->eb_mode != BBX_EB_ABS) return fail(BBX_EINVAL, "eb_mode must be REL or ABS");
  if (prm->leaf_size == 0) return fail(BBX_EINVAL, "leaf_size must be >= 1");
  if (!isfinite(eb) || !(eb > 0.0)) return fail(BBX_EINVAL, "eb must be finite and > 0");
  if (prm->tile_override != 0 && prm->tile_override != 256 && prm->tile_override != 512)
    return fail(BBX_EINVAL, "tile_override must be 0, 256 or 512");
  if (prm->ref_rule > 1) return fail(BBX_EINVAL, "ref_rule must be 0 or 1");
  if (prm->ref_mode > 1) return fail(BBX_EINVAL, "ref_mode must be 0 or 1");
  if (prm->scatter_stage > 2) return fail(BBX_EINVAL, "scatter_stage must be 0, 1 or 2");
  if (prm->level_blocks > kLevelBlocks) return fail(BBX_EINVAL, "level_blocks must be 0..4096");
  if (prm->level_pairs > 1) return fail(BBX_EINVAL, "level_pairs must be 0 or 1");
  if (prm->reduce > 2) return fail(BBX_EINVAL, "reduce must be 0, 1 or 2");
  if (prm->reduce && prm->ref_mode) return fail(BBX_EUNSUPPORTED, "the bit box reduction stores references as codes (ref_mode 0)");
  if (dims != 2 && dims != 3) return fail(BBX_EUNSUPPORTED, "dims must be 2 or 3");
  if (n >= (1ull << 32)) return fail(BBX_EUNSUPPORTED, "n must be below 2^32");
  if (prm->split_rule > 3) return fail(BBX_EINVAL, "split_rule must be 0, 1, 2 or 3");
  if (prm->split_rule && prm->ref_mode)
    return fail(BBX_EUNSUPPORTED, "split rules 1-3 store references as codes (ref_mode 0)");
  if (prm->reduce && n > 0 && split_leaf_cap(n, prm->leaf_size, prm->split_rule) >= (1ull << 31))
    return fail(BBX_EUNSUPPORTED, "the bit box reduction needs fewer than 2^31 leaves");
  return BBX_OK;
}

static bbx_status check_set(const SetIn& in) {
  bbx_status st = check_compress_args(in.n, in.dims, in.dtype, in.eb, &in.prm);
  if (st != BBX_OK) return st;
  if (in.n > 0 && !in.pos) return fail(BBX_EINVAL, "positions pointer is NULL");
  if (!in.out || ((uintptr_t)in.out & 7)) return fail(BBX_EINVAL, "output must be 8-byte aligned");
  if (in.out_cap < (size_t)kHeaderBytes) return fail(BBX_ENOSPC, "output capacity below the 128-byte header");
  return BBX_OK;
}

// Byte offsets of the batch workspace regions.
struct WsLayout {
  size_t params, sets, pre, partials, keys[2], idx[2], hist, sel, rows, cb, labels, leaves, bits, spart,
      stotal, pneed, defer, lossless, red_tq, red_taken, red_slot, red_perm, red_key, red_ctr, red_ref, red_hits,
      red_seq, split, total;
};

struct Carve {
  size_t off = 0;
  size_t take(size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  }
};

// Builds the per-set descriptors (without caller pointers when `in` lacks
// them), the launch plan and the workspace layout of a batch.
static void plan_batch(const SetIn* in, uint32_t nsets, BatchPlan* bp, std::vector<SetDesc>* descs,
                       std::vector<uint64_t>* pre, WsLayout* lay) {
  memset(bp, 0, sizeof(*bp));
  bp->nsets = nsets;
  bp->tile = in[0].prm.tile_override ? in[0].prm.tile_override : 256;
  descs->assign(nsets, SetDesc());
  uint64_t key_bytes = 0, idx_n = 0, hist_n = 0, sel_n = 0, rows_n = 0, leaves_n = 0, parts = 0;
  uint64_t cb_n = 0, lab_n = 0;
  uint64_t split_bytes = 0;
  // block target of the global levels: kSoloLevelBlocks for a set alone (a
  // larger target makes the levels' blocks too short: cosmology 2^24 1.69
  // against 2.03 ms per round trip at 4096); in a batch each set's share of
  // 4 * kLevelBlocks by particle count
  uint64_t n_total = 0;
  for (uint32_t s = 0; s < nsets; ++s) n_total += in[s].n;
  auto level_blocks = [&](uint64_t n, uint32_t cap) -> uint32_t {
    uint32_t b = (uint32_t)kSoloLevelBlocks;
    if (nsets > 1 && n_total > 0) {
      const double share = 4.0 * (double)kLevelBlocks * (double)n / (double)n_total;
      b = (uint32_t)std::min<double>((double)kLevelBlocks, std::max(1.0, std::floor(share + 0.5)));
    }
    return cap ? std::min(b, cap) : b;
  };
  std::vector<uint64_t> mm(nsets), qz(nsets), tl(nsets), bg(nsets), pm(nsets), pp(nsets);
  std::vector<uint64_t> rp(nsets, 0), rl(nsets, 0), rw(nsets, 0);
  std::vector<uint8_t> stage_seen(kMaxDepth, 0);  // a set with global level k seen
  std::vector<std::vector<uint64_t>> lv(nsets), nd(nsets);
  std::vector<std::vector<uint8_t>> lk(nsets);  // per depth: the kernel family that handles it
  for (uint32_t s = 0; s < nsets; ++s) {
    const SetIn& I = in[s];
    SetDesc& D = (*descs)[s];
    memset(&D, 0, sizeof(D));
    D.fuse_depth = D.fuse_depth4 = D.fuse_depth16 = kNoFuse;
    D.pos = I.pos;
    D.out = (uint8_t*)I.out;
    D.perm = I.d_perm;
    D.d_size = I.d_size;
    D.d_status = I.d_status;
    D.n = I.n;
    D.out_cap = I.out_cap;
    D.eb = I.eb;
    D.dims = I.dims;
    D.dtype = (uint32_t)I.dtype;
    D.layout = I.prm.layout;
    D.r = I.prm.leaf_size;
    D.ref_rule = I.prm.ref_rule;
    D.ref_mode = I.prm.ref_mode;
    D.reduce = I.prm.reduce;
    D.split = I.prm.split_rule;
    D.user_perm = seq_stream(D) ? I.d_perm : nullptr;
    // a reduce set carries source indices; its leaf stage writes them to the
    // workspace (batch_upload points perm there), the caller's perm comes last
    D.track = (I.d_perm != nullptr || I.prm.ref_mode == 1 || seq_stream(D)) ? 1u : 0u;
    D.eb_mode = I.prm.eb_mode;
    D.mbits = I.dtype == BBX_F32 ? 5u : 6u;
    const uint64_t n = I.n;
    if (n > 0 && D.split) {
      // the split-rule partition (k_split.hip) makes the leaves and their
      // boxes; the version-2 packer writes the stream
      D.geom = make_geom(n, D.r);
      D.n_leaves = split_leaf_cap(n, D.r, D.split);
      D.sp_levels = split_levels(n, D.r, D.split, D.dims);
      D.sp_off = split_bytes;
      split_bytes += align_up(sp_layout(n, D.sp_levels).total);
      mm[s] = std::min<uint64_t>((n + 2047) / 2048, kMaxMinMaxBlocks);
      qz[s] = std::min<uint64_t>((n + 1023) / 1024, 16384);
      rl[s] = D.reduce ? 1 : 0;
      rw[s] = std::max<uint64_t>(1, std::min<uint64_t>((n + 2047) / 2048, 1024));
      bp->reduce = 1;
      bp->split = 1;
      if (D.reduce) {
        if (D.n_leaves <= kRedLdsBoxes || D.split == 3) bp->red_lds_boxes = 1;
        if (D.n_leaves > kRedLdsBoxes) bp->red_global = 1;
      }
      D.mm_blocks = (uint32_t)mm[s];
      D.key_off = key_bytes;
      D.idx_off = idx_n;
      D.leaf_off = leaves_n;
      D.part_off = parts;
      D.kst = (n + 63) & ~63ull;
      key_bytes += align_up((uint64_t)D.dims * D.kst * 4);
      idx_n += (n + 63) & ~63ull;
      leaves_n += D.n_leaves;
      parts += mm[s];
    } else if (n > 0) {
      D.level_blocks = level_blocks(n, I.prm.level_blocks);
      D.geom = make_geom(n, D.r);
      D.n_leaves = D.geom.L[0][0];
      if (D.r < bp->tile) {
        D.tile_mode = 1;
        uint32_t K = 0;
        while (((n + (1ull << K) - 1) >> K) > bp->tile) ++K;
        D.gl = K;
      } else {
        D.tile_mode = 0;
        uint32_t K = 0;
        while ((n >> K) > D.r) ++K;
        D.gl = ((n + (1ull << K) - 1) >> K) <= D.r ? K : K + 1;
      }
      // paired global levels (k_pair.hip): depths 2p and 2p + 1 while both
      // use global histograms and every node of the second still splits
      if (I.prm.level_pairs == 1)
        while (2 * D.npairs + 1 < D.gl && level_kind(n, 2 * D.npairs) == kLevelGlobal &&
               level_kind(n, 2 * D.npairs + 1) == kLevelGlobal && (n >> (2 * D.npairs + 1)) > D.r)
          ++D.npairs;
      D.final_buf = D.tile_mode ? key_buf(D, D.gl) : (key_buf(D, D.gl) ^ 1);
      D.fuse_depth = fuse_depth_of(n, D.gl, D.tile_mode != 0, 2, kFuseNode);
      if (D.fuse_depth != kNoFuse)
        D.fuse_depth4 = fuse_depth_of(n, D.gl, D.tile_mode != 0, 4, 4 * kFuseNode);
      if (D.fuse_depth4 != kNoFuse) {  // only over levels of many nodes
        const uint32_t f = fuse_depth_of(n, D.gl, D.tile_mode != 0, 6, 16 * kFuseNode);
        if (f != kNoFuse && f >= 2 * D.npairs && (1ull << f) >= kFuse16Nodes) D.fuse_depth16 = f;
      }
      mm[s] = std::min<uint64_t>((n + 2047) / 2048, kMaxMinMaxBlocks);
      qz[s] = std::min<uint64_t>((n + 1023) / 1024, 16384);
      tl[s] = D.tile_mode ? (1ull << D.gl) : 0;
      bg[s] = D.tile_mode ? 0 : D.n_leaves;
      const uint64_t ref_bits = D.ref_mode ? (D.dtype == BBX_F32 ? 32u : 64u) : 30u;
      const uint64_t mw = (D.n_leaves * (uint64_t)(D.dims * (D.mbits + ref_bits)) + 63) / 64;
      pm[s] = std::max<uint64_t>(1, std::min<uint64_t>((mw + kBlock - 1) / kBlock, 1024));
      const uint64_t lpb = leaves_per_block(D.r);
      pp[s] = (D.n_leaves + lpb - 1) / lpb;
      if (D.reduce) {  // its own packing kernels; the leaf ones skip it
        pm[s] = pp[s] = 0;
        rp[s] = (D.n_leaves + kBlock - 1) / kBlock;
        rl[s] = 1;
        rw[s] = std::max<uint64_t>(1, std::min<uint64_t>((n + 2047) / 2048, 1024));
        bp->reduce = 1;
        if (D.n_leaves <= kRedLdsBoxes)
          bp->red_lds_boxes = 1;
        else
          bp->red_global = 1;
      }
      uint64_t max_nodes = 0, max_blocks = 0, bin_nodes = 0, max_lab = 0;
      for (uint32_t k = 0; k < D.gl; ++k) {
        const LevelShape sh = level_shape(n, k, D.level_blocks);
        const int kind = level_kind(n, k);
        uint8_t fam = kFamGlobal;
        if (k - D.fuse_depth < 2u) {
          fam = k == D.fuse_depth ? kFamFused : kFamNone;
          if (k == D.fuse_depth) bp->lv_fused[k] = 1;  // both levels in one pass
        } else if (k - D.fuse_depth4 < 2u) {
          fam = k == D.fuse_depth4 ? kFamFused4 : kFamNone;
          if (k == D.fuse_depth4) bp->lv_fused4[k] = 1;
        } else if (k - D.fuse_depth16 < 2u) {
          fam = k == D.fuse_depth16 ? kFamFused16 : kFamNone;
          if (k == D.fuse_depth16) bp->lv_fused16[k] = 1;
        } else if (kind == 2) {
          fam = kFamWave;
          bp->lv_wave[k] = 1;
        } else if (kind == 1) {
          fam = kFamLocal;
          bp->lv_local[k] = 1;
        } else if (pair_first(D, k))
          bp->lv_global[k] = bp->lv_pair[k] = 1;
        else if (!pair_second(D, k))
          bp->lv_global[k] = bp->lv_single[k] = 1;
        lk[s].push_back(fam);
        if (fam == kFamGlobal && sh.chunks > 256) {
          if (!pair_second(D, k)) bp->sel_wide[k] = 1;
          if (pair_first(D, k)) bp->pair_wide[k] = 1;  // the second level's selects use these chunks
        }
        if (fam == kFamGlobal) {  // by default staged only when every set's chunks are large
          const uint32_t mode = in[0].prm.scatter_stage;
          if (!stage_seen[k]) bp->scat_stage[k] = mode != 2;
          stage_seen[k] = 1;
          if (mode == 0 && sh.chunk_elems < kStageChunk) bp->scat_stage[k] = 0;
        }
        lv[s].push_back(sh.nodes * sh.chunks);
        nd[s].push_back(sh.nodes);
        if (kind == kLevelGlobal) {  // only these use selections and rows
          max_nodes = std::max(max_nodes, sh.nodes);
          max_blocks = std::max(max_blocks, sh.nodes * sh.chunks);
          max_lab = std::max(max_lab, sh.nodes * sh.chunks * (uint64_t)(sh.chunk_elems / 64));
        }
        if (kind != kLevelWave) bin_nodes = std::max(bin_nodes, sh.nodes);  // radix bins
      }
      bp->max_gl = std::max(bp->max_gl, D.gl);
      D.mm_blocks = (uint32_t)mm[s];
      D.key_off = key_bytes;
      D.idx_off = idx_n;
      D.hist_off = hist_n;
      D.hist_half = bin_nodes * kHistBins;
      D.sel_off = sel_n;
      D.sel_half = max_nodes;
      D.rows_off = rows_n * kRowStride;
      D.cb_off = cb_n;
      D.cb_half = 4 * max_blocks;  // a paired second level: two children per parent chunk
      D.lab_off = lab_n;
      D.leaf_off = leaves_n;
      D.part_off = parts;
      D.kst = (n + 63) & ~63ull;
      key_bytes += align_up((uint64_t)D.dims * D.kst * 4);
      if (I.need_idx || D.track) idx_n += (n + 63) & ~63ull;
      if (D.reduce && !(I.need_idx || D.track)) idx_n += (n + 63) & ~63ull;
      hist_n += 2 * bin_nodes * kHistBins;
      sel_n += 2 * max_nodes;
      rows_n += 2 * max_blocks;
      cb_n += 2 * D.cb_half;
      lab_n += max_lab;
      leaves_n += D.n_leaves;
      parts += mm[s];
    }
    if (D.track) bp->track = 1;
  }
  bp->total_leaves = leaves_n;
  bp->hist_entries = hist_n;
  // prefix arrays
  pre->clear();
  auto add = [&](const std::vector<uint64_t>& blocks, uint64_t* grid) -> uint64_t {
    const uint64_t off = pre->size();
    uint64_t run = 0;
    for (uint32_t s = 0; s < nsets; ++s) {
      pre->push_back(run);
      run += blocks[s];
    }
    pre->push_back(run);
    *grid = run;
    return off;
  };
  bp->o_mm = add(mm, &bp->g_mm);
  bp->o_qz = add(qz, &bp->g_qz);
  bp->o_tile = add(tl, &bp->g_tile);
  bp->o_big = add(bg, &bp->g_big);
  bp->o_pm = add(pm, &bp->g_pm);
  bp->o_pp = add(pp, &bp->g_pp);
  bp->o_rp = add(rp, &bp->g_rp);
  bp->o_rl = add(rl, &bp->g_rl);
  bp->o_rw = add(rw, &bp->g_rw);
  // Per depth and kernel family, the blocks (or node wavefronts) of the sets
  // that family handles there and none for the others, so that a launch spans
  // only its own sets' nodes; a family no set uses at a depth gets no array.
  for (uint32_t k = 0; k < bp->max_gl; ++k) {
    auto fam_add = [&](uint8_t fam, bool chunks, uint64_t* grid) -> uint64_t {
      std::vector<uint64_t> a(nsets, 0);
      bool any = false;
      for (uint32_t s = 0; s < nsets; ++s)
        if (k < lk[s].size() && lk[s][k] == fam) {
          a[s] = chunks ? lv[s][k] : nd[s][k];
          any = true;
        }
      *grid = 0;
      return any ? add(a, grid) : 0;
    };
    bp->o_lv[k] = fam_add(kFamGlobal, true, &bp->g_lv[k]);
    bp->o_nd[k] = fam_add(kFamGlobal, false, &bp->g_nd[k]);
    bp->o_lc[k] = fam_add(kFamLocal, true, &bp->g_lc[k]);
    bp->o_wv[k] = fam_add(kFamWave, false, &bp->g_wv[k]);
    bp->o_fu[k] = fam_add(kFamFused, false, &bp->g_fu[k]);
    bp->o_f4[k] = fam_add(kFamFused4, false, &bp->g_f4[k]);
    bp->o_f16[k] = fam_add(kFamFused16, false, &bp->g_f16[k]);
  }
  bp->pre_entries = pre->size();
  Carve c;
  lay->params = c.take(sizeof(DevParams) * nsets);
  lay->sets = c.take(sizeof(SetDesc) * nsets);
  lay->pre = c.take(8 * bp->pre_entries);
  lay->partials = c.take(64 * (parts + 1));
  lay->keys[0] = c.take(key_bytes);
  lay->keys[1] = c.take(key_bytes);
  lay->idx[0] = c.take(4 * idx_n);
  lay->idx[1] = c.take(4 * idx_n);
  lay->hist = c.take(4 * hist_n);
  lay->sel = c.take(sizeof(NodeSel) * sel_n);
  lay->rows = c.take(4 * kRowStride * rows_n);
  lay->cb = c.take(4 * cb_n);
  lay->labels = c.take(8 * lab_n);
  lay->leaves = c.take(sizeof(LeafRec) * leaves_n);
  lay->bits = c.take(8 * leaves_n);
  lay->spart = c.take(8 * (scan_blocks(leaves_n) + 1));
  lay->stotal = c.take(8);
  lay->pneed = c.take(4 * 4 * kMaxDepth);
  lay->defer = c.take(4 * (bp->g_tile + 1));
  lay->lossless = c.take(4 * (nsets + 1));
  const uint64_t rn = bp->reduce ? idx_n : 0, rlv = bp->reduce ? leaves_n : 0;
  lay->red_tq = c.take(16 * rn);
  lay->red_taken = c.take(rn);
  lay->red_slot = c.take(4 * rn);
  lay->red_perm = c.take(4 * rn);
  lay->red_key = c.take(8 * rlv);
  lay->red_ctr = c.take(16 * rlv);
  lay->red_ref = c.take(4 * rlv);
  lay->red_hits = c.take(4 * rlv);
  lay->red_seq = c.take(16 * rlv);
  lay->split = c.take(split_bytes);
  lay->total = c.off;
}

static Ws carve_ws(const WsLayout& L, uint8_t* base) {
  Ws w;
  w.params = (DevParams*)(base + L.params);
  w.sets = (const SetDesc*)(base + L.sets);
  w.pre = (const uint64_t*)(base + L.pre);
  w.partials = (double*)(base + L.partials);
  w.keys[0] = base + L.keys[0];
  w.keys[1] = base + L.keys[1];
  w.idx[0] = (uint32_t*)(base + L.idx[0]);
  w.idx[1] = (uint32_t*)(base + L.idx[1]);
  w.hist = (uint32_t*)(base + L.hist);
  w.sel = (NodeSel*)(base + L.sel);
  w.rows = (uint32_t*)(base + L.rows);
  w.chunk_base = (uint32_t*)(base + L.cb);
  w.labels = (uint64_t*)(base + L.labels);
  w.leaves = (LeafRec*)(base + L.leaves);
  w.leaf_bits = (uint64_t*)(base + L.bits);
  w.scan_part = (uint64_t*)(base + L.spart);
  w.scan_total = (uint64_t*)(base + L.stotal);
  w.pass_need = (uint32_t*)(base + L.pneed);
  w.tile_defer = (uint32_t*)(base + L.defer);
  w.lossless = (uint32_t*)(base + L.lossless);
  w.red_tq = (uint4*)(base + L.red_tq);
  w.red_taken = base + L.red_taken;
  w.red_slot = (uint32_t*)(base + L.red_slot);
  w.red_key = (uint64_t*)(base + L.red_key);
  w.red_ctr = (uint4*)(base + L.red_ctr);
  w.red_ref = (uint32_t*)(base + L.red_ref);
  w.red_hits = (uint32_t*)(base + L.red_hits);
  w.red_seq = (uint4*)(base + L.red_seq);
  w.split = base + L.split;
  return w;
}

static bbx_status check_batch(const SetIn* in, uint32_t nsets) {
  if (nsets == 0) return fail(BBX_EINVAL, "empty batch");
  const uint32_t tile = in[0].prm.tile_override;
  for (uint32_t s = 0; s < nsets; ++s) {
    bbx_status st = check_set(in[s]);
    if (st != BBX_OK) return fail(st, "set " + std::to_string(s) + ": " + g_err);
    if (in[s].prm.tile_override != tile) return fail(BBX_EINVAL, "all sets of a batch share one tile_override");
    if (in[s].prm.scatter_stage != in[0].prm.scatter_stage)
      return fail(BBX_EINVAL, "all sets of a batch share one scatter_stage");
  }
  return BBX_OK;
}

// Host-side check of a batch plan against what the kernels assume of it
// (bbx_plan_check).  Returns an empty string when every check holds.
static std::string check_plan(const SetIn* in, uint32_t nsets) {
  BatchPlan bp;
  std::vector<SetDesc> descs;
  std::vector<uint64_t> pre;
  WsLayout lay;
  plan_batch(in, nsets, &bp, &descs, &pre, &lay);
  auto where = [](uint32_t s, uint32_t k) {
    return "set " + std::to_string(s) + " level " + std::to_string(k) + ": ";
  };
  const uint64_t rows_total = (lay.cb - lay.rows) / (4 * kRowStride);
  for (uint32_t s = 0; s < nsets; ++s) {
    const SetDesc& D = descs[s];
    const uint64_t n = D.n;
    if (n == 0 || D.split) continue;  // a split-rule partition sizes its lists on the device
    if (D.level_blocks < 1 || D.level_blocks > kLevelBlocks) return where(s, 0) + "block target out of range";
    const uint64_t next_rows = s + 1 < nsets && descs[s + 1].n ? descs[s + 1].rows_off / kRowStride
                                                               : rows_total;
    const uint64_t rows_cap = next_rows - D.rows_off / kRowStride;
    const uint64_t bin_nodes = D.hist_half / kHistBins;
    int prev_kind = kLevelGlobal;
    uint64_t sel_need = 0;
    // set s's share of a family's grid at level k (the family's array must exist)
    auto share = [&](uint64_t off, uint64_t grid) -> uint64_t {
      if (bp.pre_entries == 0 || grid == 0) return 0;
      return pre[off + s + 1] - pre[off + s];
    };
    for (uint32_t k = 0; k < D.gl; ++k) {
      const int kind = level_kind(n, k);
      const LevelShape sh = level_shape(n, k, D.level_blocks);
      const uint64_t maxsz = (n + (1ull << k) - 1) >> k;
      if (kind < prev_kind) return where(s, k) + "level kinds are not global, then block, then wavefront";
      prev_kind = kind;
      if (sh.nodes != (1ull << k)) return where(s, k) + "node count";
      if (level_fused(D, k)) {
        const uint32_t f = k - D.fuse_depth < 2u    ? D.fuse_depth
                           : k - D.fuse_depth4 < 2u ? D.fuse_depth4
                                                    : D.fuse_depth16;
        const uint64_t cap = f == D.fuse_depth ? kFuseNode : f == D.fuse_depth4 ? 4 * kFuseNode : 16 * kFuseNode;
        if (f + 1 >= D.gl) return where(s, k) + "fused pair reaches the leaf stage";
        if (((n + (1ull << f) - 1) >> f) > cap) return where(s, k) + "fused node above its capacity";
        if (f != D.fuse_depth16 && kind != kLevelWave) return where(s, k) + "fused level is not a wavefront level";
        if (f == D.fuse_depth16 && (1ull << f) < kFuse16Nodes) return where(s, k) + "16-wavefront pair over too few nodes";
        if (f == D.fuse_depth16 && (D.fuse_depth4 == kNoFuse || f < 2 * D.npairs))
          return where(s, k) + "16-wavefront pair without a block pair below it or among paired levels";
        if (D.fuse_depth != kNoFuse && D.fuse_depth4 != kNoFuse && D.fuse_depth4 + 2 > D.fuse_depth)
          return where(s, k) + "fused pairs overlap";
        if (D.fuse_depth4 != kNoFuse && D.fuse_depth16 != kNoFuse && D.fuse_depth16 + 2 > D.fuse_depth4)
          return where(s, k) + "fused pairs overlap";
        if (k == D.fuse_depth && (!bp.lv_fused[k] || share(bp.o_fu[k], bp.g_fu[k]) != sh.nodes))
          return where(s, k) + "fused pair's grid share differs from its nodes";
        if (k == D.fuse_depth4 && (!bp.lv_fused4[k] || share(bp.o_f4[k], bp.g_f4[k]) != sh.nodes))
          return where(s, k) + "fused pair's grid share differs from its nodes";
        if (k == D.fuse_depth16 && (!bp.lv_fused16[k] || share(bp.o_f16[k], bp.g_f16[k]) != sh.nodes))
          return where(s, k) + "fused pair's grid share differs from its nodes";
        continue;
      }
      if (kind == kLevelWave) {
        if (maxsz > kWaveNode) return where(s, k) + "wavefront node above its capacity";
        if (!bp.lv_wave[k] || share(bp.o_wv[k], bp.g_wv[k]) != sh.nodes)
          return where(s, k) + "wavefront level's grid share differs from its nodes";
        continue;
      }
      // block-local and global levels count radix bins of their nodes
      if (sh.nodes > bin_nodes) return where(s, k) + "radix bins too few";
      if (kind == kLevelBlock) {
        if (sh.chunks != 1) return where(s, k) + "block-local level with more than one chunk per node";
        if (level_shape(n, k, kLocalBlocks).chunks != 1) return where(s, k) + "block-local kind";
        if (!bp.lv_local[k] || share(bp.o_lc[k], bp.g_lc[k]) != sh.nodes)
          return where(s, k) + "block-local level's grid share differs from its nodes";
        continue;
      }
      if (sh.chunk_elems == 0 || sh.chunk_elems % kGroup) return where(s, k) + "chunk not whole groups";
      if (sh.chunks * (uint64_t)sh.chunk_elems < maxsz) return where(s, k) + "chunks do not cover the node";
      if ((sh.chunks - 1) * (uint64_t)sh.chunk_elems >= maxsz) return where(s, k) + "empty chunk in the largest node";
      if (sh.nodes * sh.chunks > rows_cap) return where(s, k) + "chunk rows too few";
      if (share(bp.o_lv[k], bp.g_lv[k]) != sh.nodes * sh.chunks || share(bp.o_nd[k], bp.g_nd[k]) != sh.nodes)
        return where(s, k) + "grid share differs from the level shape";
      if (sh.chunks > 256 && !pair_second(D, k) && !bp.sel_wide[k]) return where(s, k) + "wide select not launched";
      if (pair_first(D, k)) {  // the pair's second level lives in this level's chunks
        if (k + 1 >= D.gl || level_kind(n, k + 1) != kLevelGlobal) return where(s, k) + "pair without a second global level";
        if ((n >> (k + 1)) <= D.r) return where(s, k) + "pair whose second level has leaves";
        if (!bp.lv_pair[k]) return where(s, k) + "pair not launched";
        if (sh.chunks > 256 && !bp.pair_wide[k]) return where(s, k) + "pair's wide select not launched";
        if (2 * sh.nodes * sh.chunks > rows_cap) return where(s, k) + "pair rows too few";
        if (4 * sh.nodes * sh.chunks > D.cb_half) return where(s, k) + "pair chunk bases too few";
        const uint64_t next_lab = s + 1 < nsets && descs[s + 1].n ? descs[s + 1].lab_off
                                                                  : (lay.leaves - lay.labels) / 8;
        if (sh.nodes * sh.chunks * (uint64_t)(sh.chunk_elems / 64) > next_lab - D.lab_off)
          return where(s, k) + "pair labels too few";
      } else if (!pair_second(D, k) && !bp.lv_single[k]) {
        return where(s, k) + "scatter not launched";
      }
      if (bp.scat_stage[k] && in[0].prm.scatter_stage == 0 && sh.chunk_elems < kStageChunk)
        return where(s, k) + "staged scatter on short chunks";
      sel_need = std::max(sel_need, sh.nodes);
    }
    const uint64_t next_sel = s + 1 < nsets && descs[s + 1].n ? descs[s + 1].sel_off
                                                              : (lay.rows - lay.sel) / sizeof(NodeSel);
    if (sel_need > next_sel - D.sel_off) return where(s, D.gl) + "node selections too few";
    // the leaf stage below the partition levels
    const uint64_t leafsz = (n + (1ull << D.gl) - 1) >> D.gl;
    if (D.tile_mode ? leafsz > bp.tile : leafsz > D.r) return where(s, D.gl) + "leaf stage node too large";
    if (D.gl > 0 && ((n + (1ull << (D.gl - 1)) - 1) >> (D.gl - 1)) <= (D.tile_mode ? bp.tile : D.r))
      return where(s, D.gl) + "a partition level above the leaf stage is not needed";
  }
  return std::string();
}

// A small descriptor blob travels as a kernel argument: no host-to-device
// copy, so the host never waits for the stream and the upload can be
// recorded in a graph.
constexpr uint32_t kArgBlob = 2304;  // one set at any size fits
struct ArgBlob {
  uint32_t words;
  uint32_t w[kArgBlob / 4];
};

__global__ void __launch_bounds__(kBlock) k_put_blob(ArgBlob b, uint32_t* dst) {
  for (uint32_t i = threadIdx.x; i < b.words; i += blockDim.x) dst[i] = b.w[i];
}

// Uploads descriptors and prefix arrays (stream-ordered).
static bbx_status batch_upload(const SetIn* in, uint32_t nsets, void* d_ws, size_t ws_size,
                               hipStream_t stream) {
  BatchPlan bp;
  std::vector<SetDesc> descs;
  std::vector<uint64_t> pre;
  WsLayout lay;
  plan_batch(in, nsets, &bp, &descs, &pre, &lay);
  if (!d_ws || ((uintptr_t)d_ws & 255)) return fail(BBX_EINVAL, "workspace must be 256-byte aligned");
  if (ws_size < lay.total) return fail(BBX_ENOMEM, "workspace too small: need " + std::to_string(lay.total));
  for (uint32_t s = 0; s < nsets; ++s)
    if (seq_stream(descs[s]) && descs[s].n > 0)
      descs[s].perm = (uint32_t*)((uint8_t*)d_ws + lay.red_perm) + descs[s].idx_off;
  std::vector<uint8_t> blob(lay.pre + 8 * pre.size() - lay.sets);
  memcpy(blob.data(), descs.data(), sizeof(SetDesc) * nsets);
  memcpy(blob.data() + (lay.pre - lay.sets), pre.data(), 8 * pre.size());
  if (blob.size() <= kArgBlob) {
    ArgBlob ab;
    memset(&ab, 0, sizeof(ab));
    ab.words = (uint32_t)((blob.size() + 3) / 4);
    memcpy(ab.w, blob.data(), blob.size());
    BBX_LAUNCH("upload", k_put_blob, 1, kBlock, 0, stream, ab, (uint32_t*)((uint8_t*)d_ws + lay.sets));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(BBX_EHIP, std::string("descriptor upload failed: ") + hipGetErrorString(e));
    return BBX_OK;
  }
  hipError_t e = hipMemcpyAsync((uint8_t*)d_ws + lay.sets, blob.data(), blob.size(),
                                hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return fail(BBX_EHIP, std::string("descriptor upload failed: ") + hipGetErrorString(e));
  return BBX_OK;
}

// Enqueues every kernel of the batch; no host synchronization, no copies.
static bbx_status batch_launch(const SetIn* in, uint32_t nsets, void* d_ws, size_t ws_size,
                               hipStream_t stream) {
  BatchPlan bp;
  std::vector<SetDesc> descs;
  std::vector<uint64_t> pre;
  WsLayout lay;
  plan_batch(in, nsets, &bp, &descs, &pre, &lay);
  if (!d_ws || ((uintptr_t)d_ws & 255)) return fail(BBX_EINVAL, "workspace must be 256-byte aligned");
  if (ws_size < lay.total) return fail(BBX_ENOMEM, "workspace too small: need " + std::to_string(lay.total));
  const Ws w = carve_ws(lay, (uint8_t*)d_ws);
  hipError_t e = launch_range(bp, w, stream);
  if (e == hipSuccess) e = launch_split(bp, descs.data(), w, stream);
  if (e == hipSuccess) e = launch_levels(bp, w, stream);
  if (e == hipSuccess) e = launch_leaves(bp, w, stream);
  if (e == hipSuccess) e = launch_reduce(bp, w, stream);
  if (e == hipSuccess) e = launch_pack(bp, w, stream);
  if (e != hipSuccess) return fail(BBX_EHIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
  return BBX_OK;
}

// ---------------------------------------------------------------- stream header

struct HostHeader {
  uint32_t version;
  uint64_t n_seq;
  uint64_t n, n_leaves, meta_bits, payload_bits;
  uint32_t dims, dtype, r, eb_mode, mbits, ref_mode;
  uint32_t G[3];
  double eb_user, eb_abs, eb_eff, w, inv_w, origin[3];
};

static uint64_t rd64(const uint8_t* b) {
  uint64_t v;
  memcpy(&v, b, 8);
  return v;
}
static double rdf(const uint8_t* b) {
  double v;
  memcpy(&v, b, 8);
  return v;
}

static bbx_status parse_header(const uint8_t* h, size_t bytes, HostHeader* o) {
  if (!h || bytes < (size_t)kHeaderBytes) return fail(BBX_ECORRUPT, "stream shorter than its header");
  uint32_t magic;
  memcpy(&magic, h, 4);
  uint16_t ver;
  memcpy(&ver, h + 4, 2);
  if (magic != kMagic || ver < 1 || ver > 3) return fail(BBX_ECORRUPT, "bad magic or version");
  o->version = ver;
  o->dtype = h[6];
  o->dims = h[7];
  o->n = rd64(h + 8);
  memcpy(&o->r, h + 16, 4);
  o->eb_mode = h[20];
  o->ref_mode = h[22];
  o->mbits = h[23];
  const uint32_t split = h[21];  // split rule: 1-3 only in version-2 streams
  if (o->dtype > 1 || (o->dims != 2 && o->dims != 3) || o->eb_mode > 1 || split > 3 ||
      (split && ver != 2) || h[22] > 1)
    return fail(BBX_ECORRUPT, "bad dtype, dims, eb_mode or rule fields");
  if (o->mbits != (o->dtype == 0 ? 5u : 6u) || o->r == 0 || o->n >= (1ull << 32))
    return fail(BBX_ECORRUPT, "bad width-field size, leaf size or n");
  if (ver == 3) {  // every coordinate stored as its bits: no grid, leaves or meta section
    o->eb_user = rdf(h + 24);
    o->eb_abs = rdf(h + 32);
    o->eb_eff = o->w = o->inv_w = 0.0;
    for (uint32_t d = 0; d < 3; ++d) o->origin[d] = 0.0, o->G[d] = 0;
    for (int k = 40; k < 104; ++k)
      if (h[k] != 0) return fail(BBX_ECORRUPT, "lossless stream with grid, leaf or meta fields");
    if (h[21] != 0 || h[22] != 0) return fail(BBX_ECORRUPT, "bad rule fields");
    o->n_leaves = 0;
    o->meta_bits = 0;
    o->payload_bits = rd64(h + 112);
    o->n_seq = rd64(h + 120);
    if (o->payload_bits != o->n * o->dims * (o->dtype == 0 ? 32ull : 64ull) || o->n_seq != 0)
      return fail(BBX_ECORRUPT, "lossless payload size mismatch");
    return BBX_OK;
  }
  o->eb_user = rdf(h + 24);
  o->eb_abs = rdf(h + 32);
  o->eb_eff = rdf(h + 40);
  o->w = rdf(h + 48);
  o->inv_w = rdf(h + 56);
  uint32_t sumG = 0;
  for (uint32_t d = 0; d < 3; ++d) {
    o->origin[d] = rdf(h + 64 + 8 * d);
    o->G[d] = h[88 + d];
    if (d >= o->dims && (o->G[d] != 0 || o->origin[d] != 0.0)) return fail(BBX_ECORRUPT, "unused axis fields not zero");
    if (o->G[d] > 30 || !isfinite(o->origin[d])) return fail(BBX_ECORRUPT, "bad code width or origin");
    sumG += o->G[d];
  }
  if (!isfinite(o->w) || o->w < 0.0 || !isfinite(o->inv_w) || o->inv_w < 0.0)
    return fail(BBX_ECORRUPT, "bad bin width");
  for (int k = 91; k < 96; ++k)
    if (h[k] != 0) return fail(BBX_ECORRUPT, "header padding not zero");
  o->n_leaves = rd64(h + 96);
  o->meta_bits = rd64(h + 104);
  o->payload_bits = rd64(h + 112);
  // the partition's leaf count: fixed by (n, r) and the split rule, except
  // rule 3's (at most one leaf per particle)
  const uint64_t nl = split == 3 ? o->n_leaves : (split ? split_leaf_cap(o->n, o->r, split)
                                                        : (o->n ? make_geom(o->n, o->r).L[0][0] : 0));
  if (o->n_leaves != nl || nl > o->n || (o->n > 0 && nl == 0))
    return fail(BBX_ECORRUPT, "leaf count does not match (n, r)");
  o->n_seq = rd64(h + 120);
  if (o->version == 2) {  // sequences of the bit box reduction
    if (o->ref_mode != 0) return fail(BBX_ECORRUPT, "reduced stream with stored coordinates");
    if (o->n_seq > nl || (o->n > 0 && o->n_seq == 0)) return fail(BBX_ECORRUPT, "sequence count out of range");
    if (o->meta_bits != o->n_seq * (uint64_t)(o->dims * o->mbits + sumG + 32))
      return fail(BBX_ECORRUPT, "meta size mismatch");
    if (o->payload_bits > o->n * (uint64_t)o->dims * 31u) return fail(BBX_ECORRUPT, "payload size out of range");
    return BBX_OK;
  }
  if (o->n_seq != 0) return fail(BBX_ECORRUPT, "reserved field not zero");
  const uint32_t ref_bits = o->ref_mode ? o->dims * (o->dtype == 0 ? 32u : 64u) : sumG;
  if (o->meta_bits != nl * (uint64_t)(o->dims * o->mbits + ref_bits))
    return fail(BBX_ECORRUPT, "meta size mismatch");
  if (o->payload_bits > o->n * (uint64_t)o->dims * 31u) return fail(BBX_ECORRUPT, "payload size out of range");
  return BBX_OK;
}

static uint64_t stream_bytes_of(const HostHeader& h) {
  return kHeaderBytes + ((h.meta_bits + 63) / 64) * 8 + ((h.payload_bits + 63) / 64) * 8;
}

static size_t carve_decompress(const HostHeader& h, uint8_t* base, DecompressWs* w) {
  Carve c;
  const size_t o_params = c.take(sizeof(DevParams));
  const size_t o_leaves = c.take(h.n_leaves * sizeof(LeafRec));
  const size_t o_bits = c.take(h.n_leaves * 8);
  const size_t o_sp = c.take((scan_blocks(h.n_leaves) + 1) * 8);
  const size_t o_ss = c.take(h.version == 2 ? h.n_seq * 8 : 0);
  if (w && base) {
    w->slot_start = (uint64_t*)(base + o_ss);
    w->params = (DevParams*)(base + o_params);
    w->leaves = (LeafRec*)(base + o_leaves);
    w->leaf_bits = (uint64_t*)(base + o_bits);
    w->scan_part = (uint64_t*)(base + o_sp);
  }
  return c.off;
}

static DecompressPlan plan_of(const HostHeader& h, const void* raw, uint32_t layout) {
  DecompressPlan p;
  memset(&p, 0, sizeof(p));
  memcpy(p.header.w, raw, kHeaderBytes);
  p.version = h.version;
  p.n_seq = h.n_seq;
  p.n = h.n;
  p.n_leaves = h.n_leaves;
  p.meta_bits = h.meta_bits;
  p.payload_bits = h.payload_bits;
  p.dims = h.dims;
  p.dtype = h.dtype;
  p.r = h.r;
  p.mbits = h.mbits;
  p.layout = layout;
  p.ref_mode = h.ref_mode;
  for (int d = 0; d < 3; ++d) p.G[d] = h.G[d], p.origin[d] = h.origin[d];
  p.w = h.w;
  p.inv_w = h.inv_w;
  if (h.n) p.geom = make_geom(h.n, h.r);
  return p;
}

// Bytes of the Sec. 4.2 sequence layout of a ref_mode 1 stream: per leaf the
// centre (dims * M bits), the widths (dims * mbits), the member codes and a
// 32-bit end mark, zero-padded to 8 bytes.
static uint64_t export_bytes(const HostHeader& h) {
  const uint64_t M = h.dtype == 0 ? 32 : 64;
  const uint64_t bits = h.n_leaves * (h.dims * (M + h.mbits) + 32) + h.payload_bits;
  return ((bits + 63) / 64) * 8;
}

}  // namespace bbx

using namespace bbx;

extern "C" {

size_t bbx_compress_bound(uint64_t n, uint32_t dims, bbx_dtype dtype) {
  return bbx_compress_bound_mode(n, dims, dtype, 0);
}

// Every particle is a leaf's reference (dims * (mbits + G_d) <= dims * (mbits
// + 30) meta bits, or dims * (mbits + M) with ref_mode 1) or a member (at most
// dims * 31 payload bits).
size_t bbx_compress_bound_mode(uint64_t n, uint32_t dims, bbx_dtype dtype, uint32_t ref_mode) {
  if (ref_mode > 1) return 0;
  const uint64_t mbits = dtype == BBX_F64 ? 6 : 5;
  const uint64_t ref = ref_mode ? (dtype == BBX_F64 ? 64 : 32) : 30;
  const size_t b = kHeaderBytes + 16 + ((n * dims * (mbits + ref) + 63) / 64) * 8;
  // a set stored losslessly (the grid cannot meet its bound): M bits per value
  const size_t lossless = kHeaderBytes + ((n * dims * coord_bits(dtype) + 63) / 64) * 8;
  return b > lossless ? b : lossless;
}

size_t bbx_compress_bound_params(uint64_t n, uint32_t dims, bbx_dtype dtype,
                                 const bbx_params* params) {
  if (!params || params->ref_mode > 1 || params->leaf_size == 0) return 0;
  size_t b = bbx_compress_bound_mode(n, dims, dtype, params->ref_mode);
  if (params->split_rule > 3) return 0;
  if (params->split_rule && n > 0) {
    // version 2 with one record per leaf at most (widths, codes of up to 30
    // bits, a 32-bit count), the payload's offsets at most 31 bits per axis
    const uint64_t mbits = dtype == BBX_F64 ? 6 : 5;
    const uint64_t nl = split_leaf_cap(n, params->leaf_size, params->split_rule);
    const uint64_t meta = nl * (dims * (mbits + 30) + 32), pay = n * dims * 31ull;
    const size_t v2 = kHeaderBytes + 16 + ((meta + 63) / 64) * 8 + ((pay + 63) / 64) * 8;
    return b > v2 ? b : v2;
  }
  // the bit box reduction: a 32-bit count per sequence, at most one per leaf
  if (params->reduce && n > 0) b += 4 * (size_t)make_geom(n, params->leaf_size).L[0][0] + 8;
  return b;
}

size_t bbx_compress_workspace_size(uint64_t n, uint32_t dims, bbx_dtype dtype,
                                   const bbx_params* params) {
  if (check_compress_args(n, dims, dtype, 1.0, params) != BBX_OK) return 0;
  SetIn in;
  memset(&in, 0, sizeof(in));
  in.n = n;
  in.dims = dims;
  in.dtype = dtype;
  in.eb = 1.0;
  in.prm = *params;
  in.need_idx = true;  // the caller may ask for a perm output
  BatchPlan bp;
  std::vector<SetDesc> descs;
  std::vector<uint64_t> pre;
  WsLayout lay;
  plan_batch(&in, 1, &bp, &descs, &pre, &lay);
  return lay.total;
}

bbx_status bbx_compress(const void* d_pos, uint64_t n, uint32_t dims, bbx_dtype dtype, double eb,
                        const bbx_params* params, void* d_out, size_t out_cap,
                        size_t* h_out_size, uint64_t* d_size, uint32_t* d_status,
                        uint32_t* d_perm, void* d_ws, size_t ws_size, hipStream_t stream) {
  bbx_status st = check_compress_args(n, dims, dtype, eb, params);
  if (st != BBX_OK) return st;
  SetIn in;
  in.pos = d_pos;
  in.n = n;
  in.dims = dims;
  in.dtype = dtype;
  in.eb = eb;
  in.prm = *params;
  in.out = d_out;
  in.out_cap = out_cap;
  in.d_size = d_size;
  in.d_status = d_status;
  in.d_perm = d_perm;
  in.need_idx = true;  // same plan as bbx_compress_workspace_size
  st = check_set(in);
  if (st != BBX_OK) return st;
  st = batch_upload(&in, 1, d_ws, ws_size, stream);
  if (st != BBX_OK) return st;
  st = batch_launch(&in, 1, d_ws, ws_size, stream);
  if (st != BBX_OK) return st;
  if (h_out_size) {
    DevParams hp;
    hipError_t e = hipMemcpyAsync(&hp, d_ws, sizeof(hp), hipMemcpyDeviceToHost, stream);  // params[0]
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return fail(BBX_EHIP, std::string("synchronize failed: ") + hipGetErrorString(e));
    if (hp.status != BBX_OK && hp.status != kStatusLossless) {
      const char* why = hp.status == BBX_EINVAL   ? "non-finite coordinate"
                        : hp.status == BBX_EBOUND ? "error bound too small for the input type or 30-bit codes"
                        : hp.status == BBX_ENOSPC ? "out_cap smaller than the stream"
                                                  : "device error";
      if (hp.status == BBX_EHIP && hp.diag)
        return fail(BBX_EHIP, "device consistency check " + std::to_string(hp.diag) + " failed");
      return fail((bbx_status)hp.status, why);
    }
    *h_out_size = (size_t)hp.total_bytes;
  }
  return BBX_OK;
}

static bool sets_from_abi(const bbx_set* sets, uint32_t nsets, std::vector<SetIn>* v) {
  if (!sets) return false;
  v->resize(nsets);
  for (uint32_t s = 0; s < nsets; ++s) {
    SetIn& I = (*v)[s];
    I.pos = sets[s].d_pos;
    I.n = sets[s].n;
    I.dims = sets[s].dims;
    I.dtype = (bbx_dtype)sets[s].dtype;
    I.eb = sets[s].eb;
    I.prm = sets[s].params;
    I.out = sets[s].d_out;
    I.out_cap = sets[s].out_cap;
    I.d_size = sets[s].d_size;
    I.d_status = sets[s].d_status;
    I.d_perm = sets[s].d_perm;
    I.need_idx = I.d_perm != nullptr || I.prm.ref_mode == 1;
  }
  return true;
}

size_t bbx_batch_workspace_size(const bbx_set* sets, uint32_t nsets) {
  std::vector<SetIn> v;
  if (!sets_from_abi(sets, nsets, &v) || nsets == 0) return 0;
  for (uint32_t s = 0; s < nsets; ++s)
    if (check_compress_args(v[s].n, v[s].dims, v[s].dtype, v[s].eb, &v[s].prm) != BBX_OK) return 0;
  BatchPlan bp;
  std::vector<SetDesc> descs;
  std::vector<uint64_t> pre;
  WsLayout lay;
  plan_batch(v.data(), nsets, &bp, &descs, &pre, &lay);
  return lay.total;
}

bbx_status bbx_batch_upload(const bbx_set* sets, uint32_t nsets, void* d_ws, size_t ws_size,
                            hipStream_t stream) {
  std::vector<SetIn> v;
  if (!sets_from_abi(sets, nsets, &v)) return fail(BBX_EINVAL, "sets is NULL");
  bbx_status st = check_batch(v.data(), nsets);
  if (st != BBX_OK) return st;
  return batch_upload(v.data(), nsets, d_ws, ws_size, stream);
}

bbx_status bbx_batch_launch(const bbx_set* sets, uint32_t nsets, void* d_ws, size_t ws_size,
                            hipStream_t stream) {
  std::vector<SetIn> v;
  if (!sets_from_abi(sets, nsets, &v)) return fail(BBX_EINVAL, "sets is NULL");
  bbx_status st = check_batch(v.data(), nsets);
  if (st != BBX_OK) return st;
  return batch_launch(v.data(), nsets, d_ws, ws_size, stream);
}

bbx_status bbx_compress_batch(const bbx_set* sets, uint32_t nsets, void* d_ws, size_t ws_size,
                              hipStream_t stream) {
  bbx_status st = bbx_batch_upload(sets, nsets, d_ws, ws_size, stream);
  if (st != BBX_OK) return st;
  return bbx_batch_launch(sets, nsets, d_ws, ws_size, stream);
}

bbx_status bbx_plan_check(const bbx_set* sets, uint32_t nsets) {
  std::vector<SetIn> v;
  if (!sets_from_abi(sets, nsets, &v) || nsets == 0) return fail(BBX_EINVAL, "sets is NULL or empty");
  for (uint32_t s = 0; s < nsets; ++s) {
    bbx_status st = check_compress_args(v[s].n, v[s].dims, v[s].dtype, v[s].eb, &v[s].prm);
    if (st != BBX_OK) return fail(st, "set " + std::to_string(s) + ": " + g_err);
  }
  const std::string why = check_plan(v.data(), nsets);
  if (!why.empty()) return fail(BBX_EHIP, "launch plan: " + why);
  return BBX_OK;
}

bbx_status bbx_stream_info(const void* h_header, size_t header_bytes, uint64_t* n, uint32_t* dims,
                           bbx_dtype* dtype, double* eb_abs, uint32_t* leaf_size,
                           uint64_t* n_leaves, uint64_t* stream_bytes) {
  HostHeader h;
  bbx_status st = parse_header((const uint8_t*)h_header, header_bytes, &h);
  if (st != BBX_OK) return st;
  if (n) *n = h.n;
  if (dims) *dims = h.dims;
  if (dtype) *dtype = (bbx_dtype)h.dtype;
  if (eb_abs) *eb_abs = h.eb_abs;
  if (leaf_size) *leaf_size = h.r;
  if (n_leaves) *n_leaves = h.n_leaves;
  if (stream_bytes) *stream_bytes = stream_bytes_of(h);
  return BBX_OK;
}

size_t bbx_decompress_workspace_size(const void* h_header, size_t header_bytes) {
  HostHeader h;
  if (parse_header((const uint8_t*)h_header, header_bytes, &h) != BBX_OK) return 0;
  return carve_decompress(h, nullptr, nullptr);
}

bbx_status bbx_decompress(const void* d_stream, size_t stream_size, const void* h_header,
                          void* d_pos, size_t pos_cap, bbx_layout layout, uint32_t* d_status,
                          void* d_ws, size_t ws_size, hipStream_t stream) {
  if (layout != BBX_AOS && layout != BBX_SOA) return fail(BBX_EINVAL, "layout must be AOS or SOA");
  if (!d_stream || ((uintptr_t)d_stream & 7)) return fail(BBX_EINVAL, "d_stream must be 8-byte aligned");
  if (stream_size < (size_t)kHeaderBytes) return fail(BBX_ECORRUPT, "stream shorter than its header");
  uint8_t hb[kHeaderBytes];
  if (!h_header) {
    hipError_t e = hipMemcpyAsync(hb, d_stream, kHeaderBytes, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return fail(BBX_EHIP, std::string("header copy failed: ") + hipGetErrorString(e));
    h_header = hb;
  }
  HostHeader h;
  bbx_status st = parse_header((const uint8_t*)h_header, kHeaderBytes, &h);
  if (st != BBX_OK) return st;
  if (stream_size < stream_bytes_of(h)) return fail(BBX_ECORRUPT, "stream shorter than its sections");
  const uint64_t esz = h.dtype == 0 ? 4 : 8;
  if (pos_cap < h.n * h.dims * esz) return fail(BBX_ENOSPC, "position buffer too small");
  if (h.n > 0 && (!d_pos || ((uintptr_t)d_pos & (esz - 1)))) return fail(BBX_EINVAL, "d_pos is NULL or misaligned");
  if (!d_ws || ((uintptr_t)d_ws & 255)) return fail(BBX_EINVAL, "d_ws must be 256-byte aligned");
  DecompressWs w;
  memset(&w, 0, sizeof(w));
  const size_t need = carve_decompress(h, (uint8_t*)d_ws, &w);
  if (ws_size < need) return fail(BBX_ENOMEM, "workspace too small: need " + std::to_string(need));
  const DecompressPlan p = plan_of(h, h_header, layout);
  hipError_t e = launch_decompress(p, w, (const uint8_t*)d_stream, d_pos, d_status, stream);
  if (e != hipSuccess) return fail(BBX_EHIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
  if (!d_status) {
    DevParams hp;
    e = hipMemcpyAsync(&hp, w.params, sizeof(hp), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return fail(BBX_EHIP, std::string("synchronize failed: ") + hipGetErrorString(e));
    if (hp.status != BBX_OK) return fail((bbx_status)hp.status, "stream payload fails validation");
  }
  return BBX_OK;
}

size_t bbx_export_sequences_size(const void* h_header, size_t header_bytes) {
  HostHeader h;
  if (parse_header((const uint8_t*)h_header, header_bytes, &h) != BBX_OK || h.ref_mode != 1) return 0;
  return (size_t)export_bytes(h);
}

bbx_status bbx_export_sequences(const void* d_stream, size_t stream_size, const void* h_header,
                                void* d_out, size_t out_cap, uint32_t* d_status, void* d_ws,
                                size_t ws_size, hipStream_t stream) {
  if (!d_stream || ((uintptr_t)d_stream & 7)) return fail(BBX_EINVAL, "d_stream must be 8-byte aligned");
  if (stream_size < (size_t)kHeaderBytes) return fail(BBX_ECORRUPT, "stream shorter than its header");
  uint8_t hb[kHeaderBytes];
  if (!h_header) {
    hipError_t e = hipMemcpyAsync(hb, d_stream, kHeaderBytes, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return fail(BBX_EHIP, std::string("header copy failed: ") + hipGetErrorString(e));
    h_header = hb;
  }
  HostHeader h;
  bbx_status st = parse_header((const uint8_t*)h_header, kHeaderBytes, &h);
  if (st != BBX_OK) return st;
  if (h.ref_mode != 1) return fail(BBX_EINVAL, "the sequence layout needs references stored as coordinates (ref_mode 1)");
  if (stream_size < stream_bytes_of(h)) return fail(BBX_ECORRUPT, "stream shorter than its sections");
  const uint64_t need_out = export_bytes(h);
  if (out_cap < need_out) return fail(BBX_ENOSPC, "output buffer too small: need " + std::to_string(need_out));
  if (need_out > 0 && (!d_out || ((uintptr_t)d_out & 7))) return fail(BBX_EINVAL, "d_out is NULL or not 8-byte aligned");
  if (!d_ws || ((uintptr_t)d_ws & 255)) return fail(BBX_EINVAL, "d_ws must be 256-byte aligned");
  DecompressWs w;
  memset(&w, 0, sizeof(w));
  const size_t need = carve_decompress(h, (uint8_t*)d_ws, &w);
  if (ws_size < need) return fail(BBX_ENOMEM, "workspace too small: need " + std::to_string(need));
  const DecompressPlan p = plan_of(h, h_header, BBX_AOS);
  hipError_t e = launch_export(p, w, (const uint8_t*)d_stream, d_out, d_status, stream);
  if (e != hipSuccess) return fail(BBX_EHIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
  if (!d_status) {
    DevParams hp;
    e = hipMemcpyAsync(&hp, w.params, sizeof(hp), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return fail(BBX_EHIP, std::string("synchronize failed: ") + hipGetErrorString(e));
    if (hp.status != BBX_OK) return fail((bbx_status)hp.status, "stream fails validation");
  }
  return BBX_OK;
}

// The reordered export's workspace: the decompression workspace, the plain
// layout, width histograms, per-leaf keys, (key, block) counts, the new
// order and the placed payload bits.
struct ReorderLayout {
  size_t dec, plain, whist, key, bcount, order, sbits, total;
};
static ReorderLayout reorder_layout(const HostHeader& h) {
  ReorderLayout L;
  DecompressWs w;
  Carve c;
  L.dec = c.take(carve_decompress(h, nullptr, &w));
  L.plain = c.take((size_t)export_bytes(h));
  L.whist = c.take(3 * 64 * 4);
  L.key = c.take((size_t)h.n_leaves);
  L.bcount = c.take(4 * 94 * (size_t)((h.n_leaves + kBlock - 1) / kBlock));
  L.order = c.take(4 * (size_t)h.n_leaves);
  L.sbits = c.take(8 * (size_t)h.n_leaves);
  L.total = c.off;
  return L;
}

size_t bbx_export_reordered_workspace_size(const void* h_header, size_t header_bytes) {
  HostHeader h;
  if (parse_header((const uint8_t*)h_header, header_bytes, &h) != BBX_OK || h.ref_mode != 1 ||
      h.version != 1)
    return 0;
  return reorder_layout(h).total;
}

bbx_status bbx_export_sequences_reordered(const void* d_stream, size_t stream_size,
                                          const void* h_header, void* d_out, size_t out_cap,
                                          uint32_t* h_axis_order, void* d_ws, size_t ws_size,
                                          hipStream_t stream) {
  if (!d_stream || ((uintptr_t)d_stream & 7)) return fail(BBX_EINVAL, "d_stream must be 8-byte aligned");
  if (!h_header) return fail(BBX_EINVAL, "h_header is NULL");
  HostHeader h;
  bbx_status st = parse_header((const uint8_t*)h_header, kHeaderBytes, &h);
  if (st != BBX_OK) return st;
  if (h.ref_mode != 1 || h.version != 1)
    return fail(BBX_EINVAL, "the sequence layout needs a version-1 stream with references stored as coordinates (ref_mode 1)");
  if (stream_size < stream_bytes_of(h)) return fail(BBX_ECORRUPT, "stream shorter than its sections");
  const uint64_t need_out = export_bytes(h);
  if (out_cap < need_out) return fail(BBX_ENOSPC, "output buffer too small: need " + std::to_string(need_out));
  if (need_out > 0 && (!d_out || ((uintptr_t)d_out & 7))) return fail(BBX_EINVAL, "d_out is NULL or not 8-byte aligned");
  if (!d_ws || ((uintptr_t)d_ws & 255)) return fail(BBX_EINVAL, "d_ws must be 256-byte aligned");
  const ReorderLayout L = reorder_layout(h);
  if (ws_size < L.total) return fail(BBX_ENOMEM, "workspace too small: need " + std::to_string(L.total));
  uint8_t* base = (uint8_t*)d_ws;
  DecompressWs w;
  memset(&w, 0, sizeof(w));
  carve_decompress(h, base + L.dec, &w);
  const DecompressPlan p = plan_of(h, h_header, BBX_AOS);
  uint8_t* plain = base + L.plain;
  uint32_t* whist = (uint32_t*)(base + L.whist);
  hipError_t e = launch_export(p, w, (const uint8_t*)d_stream, plain, nullptr, stream);
  if (e == hipSuccess) e = hipMemsetAsync(whist, 0, 3 * 64 * 4, stream);
  if (e == hipSuccess)
    e = launch_reorder_hist(h.n_leaves, h.dims, w, whist, base + L.key, (uint32_t*)(base + L.bcount), stream);
  uint32_t hw[3 * 64];
  DevParams hp;
  if (e == hipSuccess) e = hipMemcpyAsync(hw, whist, sizeof(hw), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipMemcpyAsync(&hp, w.params, sizeof(hp), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return fail(BBX_EHIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
  if (hp.status != BBX_OK) return fail((bbx_status)hp.status, "stream fails validation");
  // axes in ascending entropy of their widths' distribution: with the same
  // number of sequences behind every axis, descending sum of c log2 c over
  // the width counts c; equal sums keep the lower axis first
  double sclog[3] = {0, 0, 0};
  for (uint32_t d = 0; d < h.dims; ++d)
    for (int b = 0; b < 64; ++b)
      if (hw[d * 64 + b]) sclog[d] += (double)hw[d * 64 + b] * log2((double)hw[d * 64 + b]);
  uint32_t ord[3] = {0, 1, 2};
  std::stable_sort(ord, ord + h.dims, [&](uint32_t a, uint32_t b) { return sclog[a] > sclog[b]; });
  if (h_axis_order)
    for (uint32_t d = 0; d < h.dims; ++d) h_axis_order[d] = ord[d];
  e = launch_reorder_write(p, w, ord, plain, (uint8_t*)d_out, need_out / 8, base + L.key,
                           (uint32_t*)(base + L.bcount), (uint32_t*)(base + L.order),
                           (uint64_t*)(base + L.sbits), stream);
  if (e == hipSuccess) e = hipMemcpyAsync(&hp, w.params, sizeof(hp), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return fail(BBX_EHIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
  if (hp.status != BBX_OK) return fail((bbx_status)hp.status, "stream fails validation");
  return BBX_OK;
}

const char* bbx_status_str(bbx_status s) {
  switch (s) {
    case BBX_OK: return "OK";
    case BBX_EINVAL: return "EINVAL";
    case BBX_ENOSPC: return "ENOSPC";
    case BBX_ECORRUPT: return "ECORRUPT";
    case BBX_EBOUND: return "EBOUND";
    case BBX_EUNSUPPORTED: return "EUNSUPPORTED";
    case BBX_EHIP: return "EHIP";
    case BBX_ENOMEM: return "ENOMEM";
  }
  return "UNKNOWN";
}

const char* bbx_last_error(void) { return g_err.c_str(); }

void bbx_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_on = on != 0;
}

void bbx_profile_reset(void) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  prof_drain();
  g_prof.clear();
}

int bbx_profile_count(void) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  prof_drain();
  return (int)g_prof.size();
}

bbx_status bbx_profile_get(int i, const char** name, uint64_t* launches, double* total_ms) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  prof_drain();
  if (i < 0 || i >= (int)g_prof.size()) return fail(BBX_EINVAL, "profile index out of range");
  if (name) *name = g_prof[i].name.c_str();
  if (launches) *launches = g_prof[i].launches;
  if (total_ms) *total_ms = g_prof[i].ms;
  return BBX_OK;
}

}  // extern "C"

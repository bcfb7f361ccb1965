/*
 * bitbox.h -- C ABI of the MI355X (gfx950) bit-box particle compressor.
 *
 * Implements the data-parallel path of the error-bounded, bit-adaptive
 * particle-position compressor of Ren, Di, Zhang, Zhao and Guo, "An
 * Error-Bounded Lossy Compression Method with Bit-Adaptive Quantization for
 * Particle Data" (arXiv 2404.02826):
 *
 *   compress   = range and bound (Sec. 3) -> quantization into bins of width
 *                2*eb (Sec. 3, linear-scale quantization) -> k-d median
 *                partition into leaves of <= r particles (Sec. 4.1) -> per-leaf
 *                bit box: reference particle nearest the AABB centre and the
 *                per-axis widths of Eq. 2 (Sec. 4.1) -> leaf bit offsets ->
 *                bit packing (Sec. 4.2, in a structure-of-arrays layout)
 *   decompress = unpack -> dequantize to the bin centre (Sec. 3)
 *
 * All entry points are extern "C", take plain host or device pointers and
 * sizes, and never throw.  Every buffer is owned by the caller; the library
 * never allocates device memory on these paths and keeps no per-call global
 * state apart from the thread-local error message.  Calls are ordered on the
 * given HIP stream.
 *
 * Stream format v1 (little-endian), produced byte-for-byte identically to the
 * CPU oracle:
 *   [0,128)   header: magic 'BBX1' u32 | version u16 = 1 | dtype u8 | dims u8 |
 *             n u64 | r u32 | eb_mode u8 | split_rule u8 = 0 | ref_mode u8 (0, 1) |
 *             mbits u8 (5 for f32, 6 for f64: Sec. 4.2) | eb_user f64 |
 *             eb_abs f64 | eb_eff f64 | w f64 | inv_w f64 | origin[3] f64 |
 *             G[3] u8 + 5 zero bytes | n_leaves u64 | meta_bits u64 |
 *             payload_bits u64 | reserved u64 = 0
 *   meta      n_leaves fixed-stride records, leaves in depth-first order:
 *             m_d (mbits each, d < dims) then, with ref_mode 0, the
 *             reference's code q_d (G_d bits each), or with ref_mode 1 the
 *             bits of the reference's original coordinate on each axis (M =
 *             32 for f32, 64 for f64: the paper's losslessly stored centre,
 *             Sec. 4.2; its code is recomputed by the quantization of Sec. 3
 *             from origin and inv_w); zero-padded to 8 bytes
 *   payload   per leaf, every non-reference member in ascending original
 *             index, per axis the code q - q_ref + 2^(m_d - 1) in m_d bits
 *             (nothing when m_d = 0); zero-padded to 8 bytes
 *   Bit i of a section is bit (i mod 64) of its little-endian u64 word i/64.
 *
 * Decompressed order: leaves depth-first; in each leaf the reference first,
 * then the other members in ascending original index (the paper keeps all
 * particles but not their order, Sec. 2.2).  The optional perm[] output of
 * compress gives the source index of every output slot.  With ref_mode 1
 * each reference decodes to its original coordinates exactly.
 *
 * Error bound: every reconstructed coordinate satisfies |x - x_hat| <= eb_abs
 * (eb_abs = eb * Delta_max for the relative mode, Delta_max the largest
 * coordinate range over the axes, Sec. 3), including FP64 and output-type
 * rounding: the bins are 2*eb_eff wide with eb_eff = eb_abs minus a guard of
 * half an FP32 ulp of the largest magnitude (FP32 input) plus 2^-48 of it.
 */
#ifndef BITBOX_H
#define BITBOX_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BBX_OK = 0,
  BBX_EINVAL = 1,       /* bad argument, or a NaN/Inf coordinate */
  BBX_ENOSPC = 2,       /* output or position buffer too small */
  BBX_ECORRUPT = 3,     /* stream fails validation */
  BBX_EBOUND = 4,       /* eb too small for the input type, or codes would need >= 30 bits */
  BBX_EUNSUPPORTED = 5, /* dims not in {2,3}, or n >= 2^32 */
  BBX_EHIP = 6,         /* a HIP runtime call failed */
  BBX_ENOMEM = 7        /* workspace too small */
} bbx_status;

typedef enum { BBX_F32 = 0, BBX_F64 = 1 } bbx_dtype;
typedef enum { BBX_EB_REL = 0, BBX_EB_ABS = 1 } bbx_eb_mode; /* xi or epsilon, Sec. 3 */
typedef enum { BBX_AOS = 0, BBX_SOA = 1 } bbx_layout;         /* [n][dims] or [dims][n] */

/* Compression parameters.  leaf_size is r of Sec. 4.1 (a node of <= r
 * particles is not split); it changes the stream.  tile_override selects the
 * on-chip tile capacity (0 = library default); it never changes the stream.
 * ref_rule picks each leaf's reference particle (the bit box centre, Sec.
 * 4.1): 0 = the member nearest the centre of the leaf's AABB (the paper's
 * rule; squared distance in doubled code space, ties to the first member in
 * leaf order); 1 = the member whose Eq. 2 widths sum_d m_d are smallest
 * (ties to the first member), which minimises the leaf's payload bits for
 * its AABB.  Either stream decodes the same way (the reference's code is
 * stored).  ref_mode says how a leaf's meta record stores the reference:
 * 0 = its codes (G_d bits per axis); 1 = its original coordinates (32 or 64
 * bits per axis, the paper's lossless centre of Sec. 4.2), which decode
 * exactly; the other members decode identically in both modes.  ref_mode 1
 * carries source indices through the partition (as a perm output does).
 * scatter_stage says how the partition levels that use global histograms
 * store a group of members: 1 = staged in on-chip memory in output order and
 * written with coalesced stores, 2 = stored straight from the ranks, 0 = the
 * library's choice by the level's chunk size (staged from 16,384 members per
 * block); like tile_override it never changes the stream, and all sets of a
 * batch share it.  level_blocks caps the number of blocks that each of the
 * set's partition levels with global histograms is cut into (0 = the
 * library's choice: 1,024 for a set alone, the set's share of 16,384 by
 * particle count in a batch, at most 4,096; otherwise 1..4096, the smaller of
 * this and that choice); fewer
 * blocks mean longer chunks per block.  It never changes the stream.
 * reduce != 0 adds the bit box reduction of Sec. 4.1 (the while loop of
 * Alg. 1) after the bit boxes: repeatedly the remaining box with the
 * smallest key (reduce 1: the sum of its widths, as the text says; 2: the
 * sum of its box lengths, Eq. 3, as the figure caption says), ties to the
 * first leaf in depth-first order, becomes a sequence of its reference, its
 * other remaining members (ascending index) and every remaining particle of
 * other boxes that lies inside its bit box (box by box in leaf order); boxes
 * that lose particles get new bit boxes, empty ones vanish.  The stream is
 * then version 2: the header's last field holds the sequence count, a meta
 * record per sequence holds the widths, the reference's codes and a 32-bit
 * count of the other particles, the payload their codes in sequence order;
 * decompression writes the sequences in order, reference first.  Needs
 * ref_mode 0 and fewer than 2^31 leaves; its loop runs one workgroup per
 * set (a set's pops are sequential), so it suits batches of moderate sets.
 * split_rule says how the partition splits a node (Sec. 4.1 fixes "along one
 * dimension at the median" but not which dimension nor the leaf count):
 * 0 = the median along the axes in turn, halving until at most r particles
 * (the library's partition, stream version 1 unless reduce is set); 1 = the
 * median along the axis whose codes spread widest in the node (lowest axis on
 * ties); 2 = ceil(n / r) leaves of floor or ceil of n / ceil(n / r)
 * particles, leaf i holding the tree-order ranks floor(i n / b) ..
 * floor((i + 1) n / b) - 1 with b = ceil(n / r), axes in turn; 3 = the
 * midpoint split of the coders Sec. 2.2 cites: cells of the code grid
 * [0, 2^G_d) halved at their midpoints along the axes in turn (one-code-wide
 * axes skipped; a cell of one code is one leaf, however many particles),
 * until at most r particles, empty halves dropped.  Rules 1-3 write a
 * version-2 stream (one sequence per leaf, or the reduction's sequences),
 * header byte 21 holding the rule and the leaf-count field the partition's
 * leaf count; they need ref_mode 0 and run a separate, untuned partition
 * (an ablation of the reading, several times slower than rule 0).
 * level_pairs says how the partition levels with global histograms move the
 * codes: 0 = one pass per level; 1 = two levels per pass where both are
 * such levels (the second level's medians are selected over side labels of
 * the first, then one stable four-way partition moves every code to its
 * grandchild: fewer bytes, but more passes over single axes and a heavier
 * partition, slower on MI355X); it never changes the stream. */
typedef struct {
  uint32_t leaf_size;     /* r >= 1 */
  uint32_t eb_mode;       /* bbx_eb_mode */
  uint32_t layout;        /* bbx_layout of the input positions */
  uint32_t tile_override; /* 0 (= 256), 256 or 512 */
  uint32_t ref_rule;      /* 0 (AABB centre) or 1 (fewest code bits) */
  uint32_t ref_mode;      /* 0 (reference code) or 1 (reference coordinates) */
  uint32_t scatter_stage; /* 0 (by chunk size), 1 (always) or 2 (never) */
  uint32_t level_blocks;  /* 0 (library's choice) or 1..4096 */
  uint32_t reduce;        /* bit box reduction: 0 none, 1 (key: sum of widths), 2 (key: sum of lengths) */
  uint32_t split_rule;    /* 0 (median, axes in turn), 1 (widest axis), 2 (ceil(n/r) leaves), 3 (midpoint cells) */
  uint32_t level_pairs;   /* 0 (one global level per pass) or 1 (two per pass) */
} bbx_params;

/* Worst-case stream size in bytes for n particles of the given type, with
 * ref_mode 0; bbx_compress_bound_mode gives it for either ref_mode (returns
 * 0 for a ref_mode other than 0 or 1). */
size_t bbx_compress_bound(uint64_t n, uint32_t dims, bbx_dtype dtype);
size_t bbx_compress_bound_mode(uint64_t n, uint32_t dims, bbx_dtype dtype, uint32_t ref_mode);
/* The same for any parameters (the bit box reduction adds a 32-bit count
 * per sequence, at most one sequence per leaf; split rules 1-3 a record per
 * leaf with its count, rule 3 at most a leaf per particle); 0 for invalid
 * parameters. */
size_t bbx_compress_bound_params(uint64_t n, uint32_t dims, bbx_dtype dtype,
                                 const bbx_params* params);

/* Device workspace bytes needed by bbx_compress for these arguments
 * (0 on invalid arguments; bbx_last_error() says why). */
size_t bbx_compress_workspace_size(uint64_t n, uint32_t dims, bbx_dtype dtype,
                                   const bbx_params* params);

/*
 * Compress n particles.
 *   d_pos      device, n*dims values of dtype in params->layout
 *   eb         xi (relative) or epsilon (absolute), > 0 and finite
 *   d_out      device, out_cap bytes; receives the stream
 *   h_out_size host; if non-NULL the call synchronizes the stream once at the
 *              end and stores the stream length; on error the returned status
 *              says why and d_out is not written
 *   d_size     device u64 (optional); receives the stream length, or
 *              UINT64_MAX if the device detected an error (async mode)
 *   d_status   device u32 (optional); receives the bbx_status of the call
 *   d_perm     device u32[n] (optional); source index of each output slot
 *   d_ws       device workspace of ws_size >= bbx_compress_workspace_size()
 * With h_out_size == NULL nothing waits: argument errors are still returned
 * at once, data errors (NaN/Inf, eb too small, out_cap too small) appear in
 * *d_status / *d_size.
 */
bbx_status bbx_compress(const void* d_pos, uint64_t n, uint32_t dims, bbx_dtype dtype, double eb,
                        const bbx_params* params, void* d_out, size_t out_cap,
                        size_t* h_out_size, uint64_t* d_size, uint32_t* d_status,
                        uint32_t* d_perm, void* d_ws, size_t ws_size, hipStream_t stream);

/*
 * bbx_compress without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  The workspace is a static device array
 * of bbx_compress_static_limit() bytes (64 MiB) per device, allocated when
 * the library is loaded and held until the process ends; the call itself
 * allocates nothing.  A set whose bbx_compress_workspace_size() exceeds the
 * limit (about 1.97 million 3-D FP32 particles) returns BBX_ENOMEM before any
 * launch.  Every call on one device shares that device's array: calls that
 * overlap on one device (several host threads or streams) race and must be
 * serialised by the caller.  Arguments and results are those of
 * bbx_compress.
 */
size_t bbx_compress_static_limit(void);
bbx_status bbx_compress_static(const void* d_pos, uint64_t n, uint32_t dims, bbx_dtype dtype,
                               double eb, const bbx_params* params, void* d_out, size_t out_cap,
                               size_t* h_out_size, uint64_t* d_size, uint32_t* d_status,
                               uint32_t* d_perm, hipStream_t stream);

/*
 * Batched compression: many independent particle sets in one launch sequence
 * (every set is compressed exactly as bbx_compress would compress it alone,
 * byte for byte).  Each set carries its own positions, size, type, bound,
 * leaf size, layout and output; all sets of one batch share tile_override.
 */
typedef struct {
  const void* d_pos;  /* device positions of this set */
  uint64_t n;
  uint32_t dims;
  uint32_t dtype;     /* bbx_dtype */
  double eb;
  bbx_params params;
  void* d_out;        /* device, out_cap bytes, 8-byte aligned */
  size_t out_cap;
  uint64_t* d_size;   /* device u64 (optional): stream length or UINT64_MAX */
  uint32_t* d_status; /* device u32 (optional): bbx_status of this set */
  uint32_t* d_perm;   /* device u32[n] (optional): source index per output slot */
} bbx_set;

/* Device workspace bytes for a batch (0 on invalid arguments). */
size_t bbx_batch_workspace_size(const bbx_set* sets, uint32_t nsets);

/*
 * Two-part form for callers that record the launch once and replay it (HIP
 * graph capture): bbx_batch_upload copies the batch's descriptors and launch
 * tables from host memory into the workspace (one host-to-device copy on
 * `stream`; the call returns once the host data has been consumed);
 * bbx_batch_launch enqueues the kernels only (no allocation, copy or
 * synchronization), reading those descriptors.  A replay of recorded
 * launches is valid while the same workspace holds the same upload.
 * Errors of a single set (NaN/Inf, bound, capacity) go to its d_status /
 * d_size and do not affect the other sets.
 */
bbx_status bbx_batch_upload(const bbx_set* sets, uint32_t nsets, void* d_ws, size_t ws_size,
                            hipStream_t stream);
bbx_status bbx_batch_launch(const bbx_set* sets, uint32_t nsets, void* d_ws, size_t ws_size,
                            hipStream_t stream);

/* bbx_batch_upload followed by bbx_batch_launch; never waits. */
bbx_status bbx_compress_batch(const bbx_set* sets, uint32_t nsets, void* d_ws, size_t ws_size,
                              hipStream_t stream);

/* Host-only self-check of the launch plan of a batch (no device access; the
 * sets' pointers are not read): plans the sets as bbx_compress_batch would
 * and checks what the partition kernels assume of the plan (level kinds in
 * order; chunks of whole streaming groups that cover every node; one chunk
 * per node on block-local levels; enough chunk rows, node selections and
 * radix bins for every level; fused pairs and the leaf stage within their
 * node capacities).  BBX_OK, or BBX_EHIP with bbx_last_error() naming the
 * set, level and check; BBX_EINVAL for invalid arguments. */
bbx_status bbx_plan_check(const bbx_set* sets, uint32_t nsets);

/* Parses and validates a stream header (host copy of its first 128 bytes). */
bbx_status bbx_stream_info(const void* h_header, size_t header_bytes, uint64_t* n,
                           uint32_t* dims, bbx_dtype* dtype, double* eb_abs, uint32_t* leaf_size,
                           uint64_t* n_leaves, uint64_t* stream_bytes);

/* Device workspace bytes needed by bbx_decompress for the stream whose
 * header is h_header (host copy of its first 128 bytes). */
size_t bbx_decompress_workspace_size(const void* h_header, size_t header_bytes);

/*
 * Decompress a stream into d_pos (n*dims values of the stream's dtype in the
 * requested layout, pos_cap bytes).
 *   h_header   optional host copy of the first 128 stream bytes; if NULL the
 *              library copies them from d_stream (one stream synchronization)
 *   d_status   device u32 (optional).  If non-NULL the call does not wait and
 *              payload corruption found on the device is reported there; if
 *              NULL the call synchronizes at the end and returns it.
 */
bbx_status bbx_decompress(const void* d_stream, size_t stream_size, const void* h_header,
                          void* d_pos, size_t pos_cap, bbx_layout layout, uint32_t* d_status,
                          void* d_ws, size_t ws_size, hipStream_t stream);

/*
 * The sequence layout of Sec. 4.2 (figure "data layout of sequences"), for
 * tools that read the paper's format.  From a stream whose references are
 * stored as original coordinates (ref_mode 1; BBX_EINVAL otherwise), one
 * sequence per leaf in stored order: the centre (the reference's
 * coordinates, 32 or 64 bits per axis), the widths m_d (mbits each), the
 * codes of the other members (per member, per axis, m_d bits, as in the
 * stream's payload) and a 32-bit end mark of all ones.  Bit i is bit
 * (i mod 64) of little-endian u64 word i/64; the whole is zero-padded to 8
 * bytes, and its length in bits is the paper's storage-cost model with one
 * sequence per leaf.  There is no header: n, r, the bound and the origin
 * stay in the stream's header.
 *   bbx_export_sequences_size  the layout's bytes (0 for an invalid header
 *                              or ref_mode 0)
 *   d_out      device, out_cap bytes, 8-byte aligned
 *   d_ws       the decompression workspace (bbx_decompress_workspace_size)
 *   d_status   as for bbx_decompress (NULL: the call waits and returns the
 *              device's verdict on the stream)
 */
size_t bbx_export_sequences_size(const void* h_header, size_t header_bytes);
bbx_status bbx_export_sequences(const void* d_stream, size_t stream_size, const void* h_header,
                                void* d_out, size_t out_cap, uint32_t* d_status, void* d_ws,
                                size_t ws_size, hipStream_t stream);

/*
 * The sequence layout after the two reorderings of Sec. 4.2 that lower its
 * entropy before Huffman coding: sequences in ascending sum of widths (equal
 * sums keep leaf order), and in each sequence the other members in
 * ascending R-index, the members' codes concatenated with the axes in
 * ascending entropy of their width distributions (the first axis most
 * significant; axes with equal sums of c log2 c over their width counts c
 * keep their order), equal R-indices in stored order.  Each member keeps its
 * codes in axis order (x, y, z); each sequence keeps its centre, widths and
 * end mark.  The same length as bbx_export_sequences, for the same streams
 * (version 1, ref_mode 1).  h_header is required; h_axis_order (optional,
 * dims entries) receives the axis order.  The call waits (the host derives
 * the axis order from the device's width histograms); d_ws holds
 * bbx_export_reordered_workspace_size bytes (0 for an unsuitable header).
 */
size_t bbx_export_reordered_workspace_size(const void* h_header, size_t header_bytes);
bbx_status bbx_export_sequences_reordered(const void* d_stream, size_t stream_size,
                                          const void* h_header, void* d_out, size_t out_cap,
                                          uint32_t* h_axis_order, void* d_ws, size_t ws_size,
                                          hipStream_t stream);

/*
 * Huffman coding of a byte buffer: the encoding phase of Sec. 3, which the
 * paper applies to its sequence layout (Sec. 4.2; bbx_export_sequences and
 * bbx_export_sequences_reordered write that layout).  Symbols are bytes;
 * code lengths from Huffman's construction (the two lightest nodes merge
 * first; on equal weights the node created earlier, leaves in symbol order
 * before merged nodes in creation order), rebuilt from the weights halved
 * (rounded up) while a code would exceed 12 bits; canonical codes in
 * (length, symbol) order.  The input is cut into chunks of 4,096 bytes that
 * decode independently.  Stream: a 176-byte header ('BBXH', version 1, the
 * 12-bit limit, n, the chunk size, the chunk count, the payload bits, then
 * the 256 code lengths, a nibble each, low nibble for the even symbol), the
 * chunks' first bit offsets (u64 each), then the codes in input order, each
 * code's most significant bit first, bit i of the payload = bit i mod 64 of
 * its u64 word i / 64, zero-padded to 8 bytes.
 *   bbx_huffman_bound           the largest stream for n input bytes
 *   bbx_huffman_workspace_size  device workspace bytes of either call
 *   bbx_huffman_encode          d_in: n bytes (16-byte aligned); d_out
 *                               (8-byte aligned) receives the stream and
 *                               *h_out_size its length; the call waits (the
 *                               host builds the code from the device's byte
 *                               histogram)
 *   bbx_huffman_decode          h_header: a host copy of the stream's first
 *                               176 bytes (it plans the launch; the device
 *                               compares it with the stream, ECORRUPT on a
 *                               difference); d_out receives n bytes (8-byte
 *                               aligned); d_status as for bbx_decompress
 *                               (NULL: the call waits and returns the
 *                               device's verdict: lengths above 12 bits, a
 *                               Kraft sum above 1, a bit that spells no code,
 *                               or a chunk that does not end at the next one's
 *                               offset are ECORRUPT)
 */
size_t bbx_huffman_bound(uint64_t n);
size_t bbx_huffman_workspace_size(uint64_t n);
bbx_status bbx_huffman_encode(const void* d_in, uint64_t n, void* d_out, size_t out_cap,
                              size_t* h_out_size, void* d_ws, size_t ws_size, hipStream_t stream);
bbx_status bbx_huffman_decode(const void* d_stream, size_t stream_size, const void* h_header,
                              void* d_out, size_t out_cap, uint32_t* d_status, void* d_ws,
                              size_t ws_size, hipStream_t stream);

/* Short name of a status value, and the calling thread's last error message. */
const char* bbx_status_str(bbx_status status);
const char* bbx_last_error(void);

/*
 * Kernel timing.  While enabled, every kernel launch of the library is
 * bracketed by HIP events on its stream; bbx_profile_get() waits for the
 * recorded events and reports, per kernel name, the number of launches and
 * their summed duration in milliseconds.  Index i runs over 0..count-1.
 */
void bbx_profile_enable(int on);
void bbx_profile_reset(void);
int bbx_profile_count(void);
bbx_status bbx_profile_get(int i, const char** name, uint64_t* launches, double* total_ms);

#ifdef __cplusplus
}
#endif
#endif /* BITBOX_H */

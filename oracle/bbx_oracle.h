/*
 * bbx_oracle.h -- plain, single-threaded CPU oracle of the bit-box particle
 * compressor's data-parallel path (quantize -> k-d median partition -> per-leaf
 * bit box -> leaf offsets -> bit packing, and the inverse unpack/dequantize).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code, header,
 * table or helper with the HIP library; the stream format and status values
 * are the same interface, written out independently here.
 *
 * Paper: Ren, Di, Zhang, Zhao, Guo, "An Error-Bounded Lossy Compression
 * Method with Bit-Adaptive Quantization for Particle Data" (arXiv 2404.02826).
 */
#ifndef BBX_ORACLE_H
#define BBX_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status values (same numbering as the product library's ABI) */
enum {
  BBXO_OK = 0,
  BBXO_EINVAL = 1,       /* bad argument or non-finite coordinate */
  BBXO_ENOSPC = 2,       /* output buffer too small */
  BBXO_ECORRUPT = 3,     /* stream fails validation */
  BBXO_EBOUND = 4,       /* error bound too small for the input type / 30-bit codes */
  BBXO_EUNSUPPORTED = 5, /* dims not in {2,3}, n >= 2^32 */
  BBXO_ENOMEM = 7
};

/* Worst-case stream size in bytes for n particles (reference stored as its
 * code), and for a given reference storage mode (see bbxo_compress_ex). */
uint64_t bbxo_compress_bound(uint64_t n, uint32_t dims, int dtype);
uint64_t bbxo_compress_bound_mode(uint64_t n, uint32_t dims, int dtype, int ref_mode);

/*
 * Compress n particles.  pos: dtype 0 = float32, 1 = float64; layout 0 =
 * [n][dims] (AoS), 1 = [dims][n] (SoA).  eb_mode 0 = value-range relative
 * (xi), 1 = absolute (epsilon).  r = leaf capacity (>= 1).  perm (optional,
 * may be NULL, n entries): source index of each decompressed output slot.
 * On success *out_size holds the stream length in bytes.
 */
int bbxo_compress(const void* pos, uint64_t n, uint32_t dims, int dtype, int layout,
                  double eb, int eb_mode, uint32_t r,
                  uint8_t* out, uint64_t out_cap, uint64_t* out_size, uint32_t* perm);

/* As bbxo_compress, with the leaf reference rule: 0 = the member nearest the
 * AABB centre (the paper's rule, what bbxo_compress uses), 1 = the member
 * whose Eq. 2 widths against the AABB have the smallest sum; ties to the
 * first member in leaf order either way.  ref_mode selects how a meta record
 * stores the reference: 0 = its codes (G_d bits per axis, what bbxo_compress
 * uses), 1 = the bits of its original coordinates (32 or 64 per axis, the
 * paper's lossless centre of Sec. 4.2), which decode exactly. */
int bbxo_compress_ex(const void* pos, uint64_t n, uint32_t dims, int dtype, int layout,
                     double eb, int eb_mode, uint32_t r, int ref_rule, int ref_mode,
                     uint8_t* out, uint64_t out_cap, uint64_t* out_size, uint32_t* perm);

/* The bit box reduction of Sec. 4.1 (the while loop of Alg. 1) after the
 * partition and bit boxes above: repeatedly the remaining leaf with the
 * smallest key (key_rule 0: sum of widths; 1: sum of box lengths), ties to
 * the first leaf, emits a sequence of its centre, its other remaining
 * members and every remaining particle of other leaves inside its bit box;
 * leaves that lose particles get new bit boxes, empty ones vanish.  Writes
 * a version-2 stream (one meta record per sequence with a 32-bit particle
 * count); perm as for bbxo_compress.  Reference stored as its codes. */
int bbxo_compress_reduced(const void* pos, uint64_t n, uint32_t dims, int dtype, int layout,
                          double eb, int eb_mode, uint32_t r, int key_rule, uint8_t* out,
                          uint64_t out_cap, uint64_t* out_size, uint32_t* perm);

/* The partition with a chosen split rule, as an ablation of the reading of
 * Sec. 4.1: 0 = median along the axes in turn, halving until at most r
 * particles (what bbxo_compress does); 1 = median along the axis of widest
 * code extent; 2 = ceil(n / r) leaves of proportional sizes; 3 = midpoint
 * (cell) split of the code grid (Sec. 2.2's coders), empty cells dropped.
 * reduce: 0 none, 1 the reduction with key sum of widths, 2 with key sum of
 * box lengths.  ref_rule as in bbxo_compress_ex (the reduction's re-fitted
 * boxes always take rule 0).  With split_rule 0 and reduce 0 the stream is
 * bbxo_compress_ex's (version 1); otherwise version 2, one sequence per leaf
 * without the reduction, the split rule in header byte 21. */
int bbxo_compress_split(const void* pos, uint64_t n, uint32_t dims, int dtype, int layout,
                        double eb, int eb_mode, uint32_t r, int split_rule, int ref_rule,
                        int reduce, uint8_t* out, uint64_t out_cap, uint64_t* out_size,
                        uint32_t* perm);

/* Decompress a stream into pos (n*dims values of the stream's dtype). */
int bbxo_decompress(const uint8_t* stream, uint64_t size, void* pos, uint64_t pos_cap_bytes,
                    int layout);

/*
 * Stage dump for stage-by-stage parity.  Any output pointer may be NULL.
 *   q        [dims][n]  quantized codes in input order
 *   order    [n]        source index of each particle in tree (leaf) order
 *   leaf_start, leaf_size, leaf_ref (position of the reference within the leaf),
 *   leaf_m   [n_leaves][3] bit widths, leaf_bits [n_leaves] payload bits
 *   scal     [16]: eb_abs, eb_eff, w, inv_w, lo[3], hi[3], G[3] (as doubles), n_leaves
 * max_leaves bounds the leaf arrays.
 */
int bbxo_stages(const void* pos, uint64_t n, uint32_t dims, int dtype, int layout,
                double eb, int eb_mode, uint32_t r,
                uint32_t* q, uint32_t* order, uint64_t max_leaves,
                uint32_t* leaf_start, uint32_t* leaf_size, uint32_t* leaf_ref,
                uint8_t* leaf_m, uint64_t* leaf_bits, double* scal);

/* As bbxo_stages, with the leaf reference rule of bbxo_compress_ex. */
int bbxo_stages_ex(const void* pos, uint64_t n, uint32_t dims, int dtype, int layout,
                   double eb, int eb_mode, uint32_t r, int ref_rule,
                   uint32_t* q, uint32_t* order, uint64_t max_leaves,
                   uint32_t* leaf_start, uint32_t* leaf_size, uint32_t* leaf_ref,
                   uint8_t* leaf_m, uint64_t* leaf_bits, double* scal);

/* The sequence layout of Sec. 4.2 (one sequence per leaf: centre as M-bit
 * coordinates, widths, member codes, 32-bit end mark of all ones) from a
 * stream with ref_mode 1 (BBXO_EINVAL for ref_mode 0).  *out_size receives
 * the layout's length in bytes (zero-padded to 8). */
int bbxo_export_sequences(const uint8_t* stream, uint64_t size, uint8_t* out, uint64_t out_cap,
                          uint64_t* out_size);

/* The same layout after the two reorderings of Sec. 4.2: sequences in
 * ascending sum of widths, members in ascending R-index (codes concatenated
 * with the axes in ascending entropy of their widths; axis_order, optional,
 * receives that order).  Same length as the plain export. */
int bbxo_export_sequences_reordered(const uint8_t* stream, uint64_t size, uint8_t* out,
                                    uint64_t out_cap, uint64_t* out_size, uint32_t* axis_order);

/* The two steps of the R-index reordering of Sec. 4.2, on their own.
 * bbxo_axis_order_by_entropy: widths [nseq][dims] (m_d of every sequence) ->
 * order[dims], the axes in ascending entropy of their width distributions
 * (ties: lower axis first).  bbxo_r_index: the codes u[d] (m[d] bits each)
 * of one member concatenated in that order, first axis most significant;
 * returns the low 64 bits and writes the high 64 bits to *hi (may be NULL). */
void bbxo_axis_order_by_entropy(const uint32_t* widths, uint64_t nseq, uint32_t dims,
                                uint32_t* order);
uint64_t bbxo_r_index(const uint64_t* u, const uint32_t* m, uint32_t dims, const uint32_t* order,
                      uint64_t* hi);

/* Huffman coding of bytes (the encoding phase of Sec. 3 applied to the
 * sequence layout of Sec. 4.2): code lengths of Huffman's construction
 * (ties: the earlier node; rebuilt from halved weights until no code is
 * longer than 12 bits), canonical codes, chunks of 4,096 input bytes with
 * their first bit offsets stored.  The stream layout is in bbx_oracle.c. */
void bbxo_huffman_lengths(const uint64_t* counts, uint32_t* len);
uint64_t bbxo_huffman_bound(uint64_t n);
int bbxo_huffman_encode(const uint8_t* in, uint64_t n, uint8_t* out, uint64_t out_cap,
                        uint64_t* out_size);
int bbxo_huffman_decode(const uint8_t* stream, uint64_t size, uint8_t* out, uint64_t out_cap,
                        uint64_t* out_n);

/* Number of leaves of the size-only recursion for n particles, capacity r. */
uint64_t bbxo_leaf_count(uint64_t n, uint32_t r);

/* Eq. 2 of the paper in its integer form: bits for a largest offset D. */
uint32_t bbxo_bits_for_offset(uint64_t D);

#ifdef __cplusplus
}
#endif
#endif

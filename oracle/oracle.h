/*
 * RLFC reference oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, deliberately unoptimised CPU implementation of what the RLFC
 * method computes (Pratapa & Manocha, "RLFC: Random Access Light Field
 * Compression using Key Views and Bounded Integer Sequence Encoding", I3D'19,
 * arXiv 1805.06019).  It exists to check the HIP library against; only the
 * test-suite, the package smoke check and the benchmark's CPU-baseline leg may
 * load it.  It shares no code, header, table or helper with the library in
 * paper_1805_06019_amd/.
 *
 * Where the paper is silent the oracle follows the readings listed in the
 * design notes (C1..C24); each function names the paper passage it follows.
 *
 * Parity status: the integer encode/decode, BISE packing, YCoCg-R and the
 * renderer are pinned by tests/test_oracle_*.py.  Parity of the quantiser
 * against the paper's own quantiser (its supplementary Section 3, not
 * available) and of bpp/PSNR against the paper's tables is UNPINNED: the
 * paper's datasets, quantiser details and JPEG2000 coder are not available.
 */
#ifndef RLFC_ORACLE_H
#define RLFC_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_LEVELS 6

/* Encoding parameters (Sec. 3.1-3.3, Alg. 1 "enc"). */
typedef struct {
  int32_t grid_u, grid_v;          /* views per row (u), rows of views (v) */
  int32_t width, height;           /* pixels per view */
  int32_t block;                   /* B in {2,4,8} */
  int32_t levels;                  /* L >= 1, tree height incl. level 0 */
  int32_t cluster[ORC_MAX_LEVELS]; /* cluster side c_l stored at [l-1], l=1..L-1 */
  int32_t pix_threshold;           /* T_pix >= 0 */
  int32_t blk_threshold;           /* T_blk >= 0 */
  int32_t quant_bits;              /* q in [0,4] */
  uint32_t range_mask;             /* allowed BISE range codes (bit k); 0 = all */
} orc_params;

/* Derived geometry. */
typedef struct {
  int32_t wp, hp;                  /* padded width/height */
  int32_t nbx, nby, nb;            /* blocks per row, per column, total */
  int32_t ng;                      /* groups = 3 * nb */
  int32_t n_srv, n_top;            /* SRV nodes (levels 0..L-2), top RKV nodes */
  int32_t lu[ORC_MAX_LEVELS], lv[ORC_MAX_LEVELS]; /* grid size per level */
} orc_geom;

/* Status codes. */
#define ORC_OK 0
#define ORC_E_INVALID (-1)
#define ORC_E_CORRUPT (-2)
#define ORC_E_NOMEM (-3)
#define ORC_E_RANGE (-5)

int orc_geometry(const orc_params *p, orc_geom *g);

/* Lossless YCoCg-R (Sec. 4, colour decorrelation): n pixels, interleaved. */
void orc_ycocg_forward(const uint8_t *rgb, int64_t n, int16_t *ycocg);
void orc_ycocg_inverse(const int16_t *ycocg, int64_t n, uint8_t *rgb_clamped);

/* BISE (Sec. 3.3): range code -> bit size of a block of S values. */
int orc_bise_range(int code, int *kind, int *m, int *n_values_bound);
int orc_bise_bits(int code, int S);
int orc_bise_encode(const uint16_t *vals, int S, int code, uint32_t *words, int64_t bitpos);
int orc_bise_decode(const uint32_t *words, int64_t bitpos, int S, int code, uint16_t *vals);

int32_t orc_zigzag(int32_t v);
int32_t orc_unzigzag(int32_t z);
int32_t orc_quantize(int32_t r, int q);

/* Tree tables (Sec. 3.4 BFS linearisation): for every view vi and level
 * l = 0..L-2 the SRV index of the view's ancestor at level l; root[vi] is the
 * top-level node.  srv_path is [U*V][L-1]. */
int orc_tree_tables(const orc_params *p, int32_t *srv_path, int32_t *root);

/* Bottom-up RKV tree (Sec. 3.1, eqs. 1-2) on YCoCg planes.  out receives
 * levels 0..L-1 back to back, each [n_l][3][hp][wp] int32. */
int orc_rkv_tree(const uint8_t *rgb, const orc_params *p, int32_t *out);

/* CompressLFI (Alg. 1).  *out is malloc'd (free with orc_free).  If r0 is not
 * NULL it receives the encoder's closed-loop level-0 reconstruction,
 * [U*V][3][hp][wp] int16.  If ycocg is not NULL it receives the padded YCoCg
 * planes of the input in the same layout.  hist (26 entries, optional)
 * receives the per-range-code block counts. */
int orc_encode(const uint8_t *rgb, const orc_params *p, uint8_t **out, int64_t *bytes,
               int16_t *r0, int16_t *ycocg, int64_t *hist);

/* Per-block encoder control.  Threshold classes 0..8: pixel threshold 0, 2,
 * 3, 4, 5, 6, 8, 12, 16, then the quantiser, the block stored if a value is
 * nonzero; class 9: the block dropped.  Range classes: BISE codes 0..25, 26 =
 * absent.  SEARCH takes, per (node, block, channel), the class of least
 * w_c * SSE * 2^16 + lambda_q16 * rate (w = 6 for Y, 1 for Co, Cg; rate = 5
 * + payload bits, 0 when absent; the first class wins ties) with the
 * smallest allowed range.  TABLE applies given classes, the values limited
 * to the given range's bound and stored with that code.  Rows: levels L-2
 * down to 0, node (row-major), block, channel.  features_out gets 16 floats
 * per row: level/4, [c == Y], log2(1+mean|r|)/8, log2(1+max|r|)/8,
 * log2(1+var|r|)/16, fractions of |r| >= 2, 4, 8, 16, log2(1+mean
 * horizontal |dp|)/8, log2(1+mean vertical |dp|)/8, log2(1+max|dp|)/8,
 * log2(1+var p)/16, q/4, log2(1+lambda_q16/2^16)/24, B/8 (r = block -
 * parent reconstruction p).  The pixel and block thresholds of the
 * parameters are used by GLOBAL only. */
#define ORC_CTL_GLOBAL 0
#define ORC_CTL_SEARCH 1
#define ORC_CTL_TABLE 2
typedef struct {
  int32_t mode;
  int64_t lambda_q16;
  const int8_t *classes_in, *ranges_in;  /* TABLE */
  int8_t *classes_out, *ranges_out;      /* may be NULL */
  float *features_out;                   /* may be NULL */
} orc_control;
int orc_encode_ctl(const uint8_t *rgb, const orc_params *p, orc_control *ctl, uint8_t **out, int64_t *bytes,
                   int16_t *r0_out, int16_t *ycocg_out, int64_t *hist);
void orc_free(void *ptr);

/* Header of a stream. */
int orc_read_header(const uint8_t *stream, int64_t bytes, orc_params *p, orc_geom *g);

/* DecompressLFIBlock (Alg. 2): the three channels of block b of view vi,
 * out is [3][B*B] int16. */
int orc_decode_block(const uint8_t *stream, int64_t bytes, int32_t vi, int32_t b, int16_t *out);

/* orc_decode_block for each of n requests req[2i] = view, req[2i+1] = block in
 * turn, block i into out + 3 B^2 i (a loop for timing and parity runs; no
 * arithmetic of its own). */
int orc_decode_requests(const uint8_t *stream, int64_t bytes, int64_t n, const int32_t *req, int16_t *out);

/* Progressive decompression (Sec. 3.6): the traversal of orc_decode_block
 * stopped at tree level `level` (0 = the view, L-1 = its key view). */
int orc_decode_block_level(const uint8_t *stream, int64_t bytes, int32_t vi, int32_t b, int32_t level,
                           int16_t *out);

/* Whole light field, group by group (Sec. 3.5), for blocks [b0, b1).
 * out is [U*V][3][hp][wp] int16. */
int orc_decode_all(const uint8_t *stream, int64_t bytes, int32_t b0, int32_t b1, int16_t *out);

/* Novel-view rendering (Sec. 3.6) by quadrilinear interpolation over a decoded
 * light field lf [U*V][3][hp][wp]; views [n][4] = (u, v, s, t);
 * out [n][3][ho][wo] RGB / 255. */
int orc_render(const int16_t *lf, int32_t U, int32_t V, int32_t W, int32_t H, int32_t wp,
               int32_t hp, const float *views, int32_t n, int32_t wo, int32_t ho, float *out);
/* orc_render refocused at disparity d: source camera (iu, jv) sampled at
 * (sx + d (iu - u), ty + d (jv - v)), (u, v) clamped to the grid. */
int orc_render_focal(const int16_t *lf, int32_t U, int32_t V, int32_t W, int32_t H, int32_t wp, int32_t hp,
                     const float *views, int32_t n, int32_t wo, int32_t ho, float d, float *out);

/* PSNR_YCoCg (eqs. 4-5), averaged over the views.  Both inputs
 * [U*V][3][hp][wp]; only the W x H area counts. */
double orc_psnr(const int16_t *ref, const int16_t *dec, int32_t nviews, int32_t W, int32_t H,
                int32_t wp, int32_t hp);

#ifdef __cplusplus
}
#endif
#endif

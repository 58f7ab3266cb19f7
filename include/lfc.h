/*
 * lfc.h -- C ABI of liblfc.so, an MI355X (gfx950) implementation of the
 * decode-and-render path of RLFC (Pratapa & Manocha, "RLFC: Random Access
 * Light Field Compression using Key Views and Bounded Integer Sequence
 * Encoding", I3D 2019, arXiv 1805.06019).
 *
 * Conventions for every call:
 *  - Pointers prefixed d_ are device pointers (hipMalloc'd or torch CUDA
 *    tensors) on the current device; every other pointer is host memory.
 *  - The caller owns every buffer it passes.  Output buffers must not alias
 *    inputs.
 *  - Every call returns an lfc_status; on a non-OK status the call has no
 *    effect on its outputs (host-side checks happen before any launch) and
 *    lfc_last_error() returns a message (thread-local).  No C++ exception
 *    crosses this interface.
 *  - Device work is enqueued on the stream argument and the call returns
 *    without waiting, except lfc_open and lfc_check, which synchronise it.
 *  - All multi-byte integers of the stream format are little-endian.
 */
#ifndef LFC_H
#define LFC_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LFC_OK = 0,
  LFC_E_INVALID = -1,      /* bad argument (null pointer, size, layout, parameter) */
  LFC_E_CORRUPT = -2,      /* stream fails validation */
  LFC_E_NOMEM = -3,        /* host or device allocation failed */
  LFC_E_HIP = -4,          /* a HIP runtime call or kernel launch failed */
  LFC_E_RANGE = -5,        /* a residual needs a BISE range above 4096 values */
  LFC_E_UNSUPPORTED = -6   /* valid request the library cannot serve */
} lfc_status;

#define LFC_MAX_LEVELS 6

/*
 * Encoding parameters -- the "enc" argument of CompressLFI (Alg. 1).
 *  grid_u, grid_v  views per row (u, the column index) and rows of views (v);
 *                  view index vi = v * grid_u + u.  1..4096 each.
 *  width, height   pixels per view, 1..65536 each.
 *  block           B, side of the square residual blocks (Sec. 3.2): 2, 4 or 8.
 *  levels          L, tree height counting the original views as level 0
 *                  (Sec. 3.1, Table 2): 1..6.  Level L-1 holds the stored
 *                  key views (RKV); levels 0..L-2 hold residual views (SRV).
 *  cluster[l-1]    side c_l of the square clusters that group level l-1 into
 *                  level l (eq. 1), l = 1..L-1; 2..8.  Clusters tile the grid
 *                  from (0,0) and are truncated at its edges.
 *  pix_threshold   residual samples with |r| below it are zeroed (Sec. 3.2).
 *  blk_threshold   blocks whose sum of |r| is not above it are dropped (Sec. 3.2).
 *  quant_bits      q: kept residuals are quantised with step 2^q, 0..4 (Sec. 3.2).
 *  range_mask      allowed BISE range codes, bit k for code k (0..25); 0 = all.
 */
typedef struct {
  int32_t grid_u, grid_v;
  int32_t width, height;
  int32_t block;
  int32_t levels;
  int32_t cluster[LFC_MAX_LEVELS];
  int32_t pix_threshold;
  int32_t blk_threshold;
  int32_t quant_bits;
  uint32_t range_mask;
} lfc_params;

/*
 * A novel camera (Sec. 3.6): (u, v) is a position on the camera plane in
 * grid units (u along a row of views, 0..grid_u-1; values outside are
 * clamped); (s, t) pans the image plane by that many source pixels.
 */
typedef struct {
  float u, v, s, t;
} lfc_view;

/* Opaque handle: one compressed light field resident in device memory. */
typedef struct lfc_lf lfc_lf;

/* Facts about an opened light field. */
typedef struct {
  lfc_params params;
  int32_t padded_width, padded_height;   /* width, height rounded up to B */
  int32_t n_blocks;                      /* NB = (padded_width/B)*(padded_height/B) */
  int32_t n_groups;                      /* 3*NB: one per (spatial block, channel) */
  int32_t n_srv;                         /* residual-view nodes in the tree */
  int32_t n_top;                         /* stored key views */
  uint64_t stream_bytes;                 /* size of the stream it was opened from */
  uint64_t device_bytes;                 /* device memory held by the handle */
  uint64_t present_blocks;               /* stored residual blocks over all groups */
} lfc_info_t;

enum { LFC_LAYOUT_BLOCKS = 0, LFC_LAYOUT_IMAGES = 1 };

/*
 * CompressLFI (Alg. 1; Sec. 3.1-3.4), on the host.
 *  rgb      host, uint8 [grid_v][grid_u][height][width][3], RGB.
 *  p        parameters as above.
 *  *stream_out receives a library-allocated host buffer holding the stream
 *           (header, RKVStream, BlockOffsets, SRVStream); free it with
 *           lfc_free.  *bytes_out receives its size.
 * Errors: LFC_E_INVALID (null pointer, parameter out of range),
 * LFC_E_RANGE (a residual block needs more than 4096 BISE values, or a
 * reconstruction leaves int16), LFC_E_NOMEM.
 */
lfc_status lfc_encode(const uint8_t *rgb, const lfc_params *p, void **stream_out,
                      size_t *bytes_out);

/* Quality and rate of an encoding, from the encoder's own reconstruction
 * (which every decode reproduces exactly). */
typedef struct {
  double psnr;             /* PSNR_YCoCg of eq. 4 from eq. 5 (peak 255, 100 dB cap), mean over views */
  double psnr_y, psnr_co, psnr_cg;  /* per-channel PSNR, mean over views */
  uint64_t present_blocks; /* stored residual blocks */
  uint64_t code_hist[26];  /* stored residual blocks per BISE range code */
  uint64_t stream_bytes;   /* size of the stream */
} lfc_encode_stats;

/*
 * lfc_encode that also reports quality and rate (Sec. 4, eqs. 4-5), for
 * choosing thresholds.  stream_out and bytes_out may both be NULL to get the
 * statistics only; stats may be NULL.  Errors as lfc_encode.
 */
lfc_status lfc_encode_ex(const uint8_t *rgb, const lfc_params *p, void **stream_out, size_t *bytes_out,
                         lfc_encode_stats *stats);

/*
 * Learned encoder control.  The paper's encoder applies one pixel threshold
 * and one block-energy threshold to every residual block (Sec. 3.2) and
 * names the lack of finer control as a limitation (Sec. 5).  Here each
 * residual block (node, spatial block, channel: a control row) gets its own
 * decision; the decoder is unchanged, since the stream carries only the
 * stored values and their range codes.
 *
 * Threshold classes 0..8 apply the pixel threshold 0, 2, 3, 4, 5, 6, 8, 12 or
 * 16 (residuals of smaller magnitude become 0), then the quantiser; the
 * block is stored if a value is nonzero.  Class 9 (LFC_CTL_DROP) drops it.
 * Range classes are the BISE range codes 0..25, or 26 (LFC_CTL_ABSENT).
 *
 * Modes (params' pix_threshold and blk_threshold are used by GLOBAL only):
 *  LFC_CTL_GLOBAL  the paper's global thresholds (= lfc_encode_ex).
 *  LFC_CTL_SEARCH  exhaustive search: per row, the threshold class of least
 *                  cost w_c * SSE * 2^16 + lambda_q16 * rate, where SSE is
 *                  the squared error of the reconstructed block against the
 *                  block being coded, w_c = 6 for Y and 1 for Co and Cg (the
 *                  weights of eq. 4), rate = 5 + BISE payload bits (0 when
 *                  absent); ties go to the lower class.  The block takes the
 *                  smallest allowed range holding its values.
 *  LFC_CTL_TABLE   replays classes[] and ranges[] (e.g. those an earlier
 *                  call used): the threshold class, then the values clamped
 *                  into the given range's bound and stored with that range
 *                  code (absent if none is nonzero, or if the range class is
 *                  26).
 *  LFC_CTL_MLP     a per-block network (lfc_mlp_infer, on the GPU, weights
 *                  d_mlp) predicts both classes from the row's 16 features;
 *                  they are applied as in TABLE (a range the mask excludes
 *                  is replaced by the values' own range).  Rows whose top
 *                  threshold-class probability is below min_confidence, or
 *                  whose prediction would leave int16, fall back to the
 *                  search (counted in fallbacks).
 * Rows are ordered by level from L-2 down to 0, then node (row-major in the
 * level's grid), spatial block, channel; lfc_control_rows gives the count.
 * The features of a row (float32, from the residuals v = block - parent
 * reconstruction and the parent reconstruction p): level/4, [channel is Y],
 * log2(1+mean|v|)/8, log2(1+max|v|)/8, log2(1+var|v|)/16, fractions of |v|
 * at least 2, 4, 8 and 16, log2(1+mean horizontal |dp|)/8, log2(1+mean
 * vertical |dp|)/8, log2(1+max |dp|)/8, log2(1+var p)/16, quant_bits/4,
 * log2(1+lambda)/24 with lambda = lambda_q16/2^16, block/8.
 */
enum { LFC_CTL_GLOBAL = 0, LFC_CTL_SEARCH = 1, LFC_CTL_TABLE = 2, LFC_CTL_MLP = 3 };
#define LFC_CTL_CLASSES 10
#define LFC_CTL_DROP 9
#define LFC_CTL_RANGES 27
#define LFC_CTL_ABSENT 26
#define LFC_CTL_FEATURES 16
typedef struct {
  int32_t mode;
  float min_confidence;      /* MLP: search below this top probability (0: never) */
  int64_t lambda_q16;        /* rate weight * 2^16, 0..2^52 (SEARCH, MLP, features) */
  const void *d_mlp;         /* MLP: device weights, LFC_MLP_PARAMS bf16 */
  hipStream_t stream;        /* MLP: stream of the inference launches */
  int64_t rows;              /* length of every array below that is given */
  int8_t *classes;           /* TABLE: in; else out (may be NULL): threshold class used */
  int8_t *ranges;            /* TABLE: in; else out (may be NULL): range class used */
  float *features;           /* out (may be NULL): [rows][16] */
  int8_t *search_classes;    /* out (may be NULL): the search's threshold class */
  int8_t *search_ranges;     /* out (may be NULL): the search's range class */
  int64_t fallbacks;         /* out: rows the search decided in MLP mode */
} lfc_control;

/* Control rows of an encoding: sum over levels 0..L-2 of nodes * NB * 3;
 * -1 for invalid parameters. */
int64_t lfc_control_rows(const lfc_params *p);

/*
 * lfc_encode_ex under a control mode.  Host memory in and out; MLP mode also
 * runs the network on the current device, on ctl->stream, and blocks until
 * it is done.
 * Errors: LFC_E_INVALID (null pointer, unknown mode, lambda out of range,
 * rows mismatch, TABLE without both tables or with an entry out of range or
 * a range the mask excludes, MLP without weights, GLOBAL with tables),
 * LFC_E_RANGE (as lfc_encode; in TABLE mode also a reconstruction leaving
 * int16), LFC_E_NOMEM, LFC_E_HIP (MLP inference).
 */
lfc_status lfc_encode_ctl(const uint8_t *rgb, const lfc_params *p, lfc_control *ctl, void **stream_out,
                          size_t *bytes_out, lfc_encode_stats *stats);

/*
 * The per-block network: 16 features -> 64 ReLU -> 64 ReLU -> 37 logits
 * (10 threshold classes, then 27 range classes).  Parameters, in this
 * order: W1[64][16], b1[64], W2[64][64], b2[64], W3[37][64], b3[37]
 * (LFC_MLP_PARAMS values).  Inference keeps them as bfloat16 and
 * accumulates in float32; training keeps float32 master weights and Adam
 * moments and re-rounds the bfloat16 copy after each update.
 */
#define LFC_MLP_PARAMS 7653

/*
 * Inference over n feature rows (device float32 [n][16], 16-byte aligned): per row the
 * argmax of each head (ties to the lower class) into d_cls and d_rng
 * (int8 [n]), the threshold head's top softmax probability into d_conf
 * (float [n], may be NULL) and the 37 logits into d_logits (float [n][37],
 * may be NULL).  d_w: device bf16 [LFC_MLP_PARAMS].
 * Errors: LFC_E_INVALID (null pointer, n < 0), LFC_E_HIP.
 */
lfc_status lfc_mlp_infer(const uint16_t *d_w, const float *d_x, int64_t n, int8_t *d_cls, int8_t *d_rng,
                         float *d_conf, float *d_logits, hipStream_t s);

/*
 * lfc_mlp_infer at a chosen precision.  LFC_MLP_FP32: float32 activations
 * (= lfc_mlp_infer).  LFC_MLP_BF16: the three layers on the matrix cores
 * (bf16 x bf16 products, float32 accumulation), the inputs and the two
 * hidden layers' outputs rounded to bf16 (to nearest, ties to even); d_w must
 * then be 16-byte aligned.  Errors: as lfc_mlp_infer, plus LFC_E_INVALID
 * (unknown precision, misaligned weights).
 */
enum { LFC_MLP_FP32 = 0, LFC_MLP_BF16 = 1 };
lfc_status lfc_mlp_infer_ex(const uint16_t *d_w, const float *d_x, int64_t n, int8_t *d_cls, int8_t *d_rng,
                            float *d_conf, float *d_logits, int32_t precision, hipStream_t s);

/*
 * Mean gradient over a batch of n rows of the loss cross-entropy(threshold
 * head, d_cls) + cross-entropy(range head, d_rng), at the bf16 weights d_w.
 * d_part: device float [ceil(n/128)][LFC_MLP_PARAMS] scratch (per-workgroup
 * partial sums); d_grad: device float [LFC_MLP_PARAMS] out; d_loss: device
 * float [1] out, the mean loss.  Labels outside 0..9 / 0..26 are errors
 * reported by a zero-gradient row and a loss of NaN.
 * Errors: LFC_E_INVALID (null pointer, n < 1), LFC_E_HIP.
 */
lfc_status lfc_mlp_grad(const uint16_t *d_w, const float *d_x, const int8_t *d_cls, const int8_t *d_rng, int32_t n,
                        float *d_part, float *d_grad, float *d_loss, hipStream_t s);

/*
 * One Adam step (bias-corrected, step >= 1) on the float32 master weights
 * d_master with moments d_m, d_v (device float [LFC_MLP_PARAMS] each) and
 * gradient d_grad, then d_w = the master rounded to bfloat16 (to nearest,
 * ties to even).  Errors: LFC_E_INVALID (null pointer, step < 1), LFC_E_HIP.
 */
lfc_status lfc_mlp_adam(float *d_master, uint16_t *d_w, float *d_m, float *d_v, const float *d_grad, int32_t step,
                        float lr, float beta1, float beta2, float eps, hipStream_t s);

/*
 * lfc_encode_ex on the GPU (the global thresholds of the parameters):
 * level 0, the key-view filters, the closed-loop residual levels and the
 * packing of every group run as kernels on stream s; the host turns the
 * group sizes into offsets and assembles the stream.  The stream and the
 * statistics equal lfc_encode_ex's byte for byte.
 *  d_rgb  device uint8 [grid_v][grid_u][height][width][3] (as lfc_encode).
 * Blocks until done.  Device memory for the tree's levels and tables is
 * allocated and freed by the call.
 * Errors: as lfc_encode, plus LFC_E_INVALID (d_rgb not device memory of that
 * size), LFC_E_NOMEM (device), LFC_E_HIP.
 */
lfc_status lfc_encode_gpu(const uint8_t *d_rgb, const lfc_params *p, void **stream_out, size_t *bytes_out,
                          lfc_encode_stats *stats, hipStream_t s);

/* Frees a buffer returned by lfc_encode.  NULL is ignored. */
void lfc_free(void *ptr);

/*
 * Checks a stream on the host without touching a device: header, section
 * sizes, monotone offsets, every group's bitmap, range codes and payload
 * length, and every BISE digit field.  p_out (may be NULL) receives the
 * stream's parameters.  Errors: LFC_E_INVALID (null pointer),
 * LFC_E_CORRUPT.
 */
lfc_status lfc_validate(const void *stream, size_t bytes, lfc_params *p_out);

/*
 * Decoder initialisation (Alg. 2 "Initialization"; Sec. 3.5, which computes
 * block and parent locations once at start-up).  Validates the stream as
 * lfc_validate does, builds the per-group block directory and the tree
 * tables, copies everything to the current device on stream s and waits for
 * the copies.  The host stream may be freed after the call returns.
 * *out receives the handle.  Errors: LFC_E_INVALID, LFC_E_CORRUPT,
 * LFC_E_NOMEM, LFC_E_HIP.
 */
lfc_status lfc_open(const void *stream, size_t bytes, hipStream_t s, lfc_lf **out);

/*
 * lfc_open with explicit settings of the handle (cfg NULL: the defaults).
 *  tile_blocks  capacity, in stored residual blocks, of the compact tile the
 *               whole-field decode fills per chunk of a strip (Sec. 3.5-3.6:
 *               blocks decode in parallel; a chunk's blocks are decoded once
 *               each, then gathered).  0: the default (2048 / 1024 / 256 for
 *               B = 2 / 4 / 8); else a multiple of 8 in 512/B..2048.  It
 *               changes the launch shape only: decoded samples do not depend
 *               on it.  lfc_tune_decode measures the choice.
 * Errors: as lfc_open, plus LFC_E_INVALID (tile_blocks out of range).
 */
typedef struct {
  int32_t tile_blocks;
} lfc_open_config;
lfc_status lfc_open_ex(const void *stream, size_t bytes, const lfc_open_config *cfg, hipStream_t s,
                       lfc_lf **out);

/* Fills *info.  Errors: LFC_E_INVALID. */
lfc_status lfc_info(const lfc_lf *lf, lfc_info_t *info);

/*
 * LDS words the whole-field decode needs to stage each strip (64/B blocks of
 * one block row and channel, strips ordered channel, block row, strip):
 * need[2i] = its groups plus its part of the decode schedule, need[2i+1] =
 * the schedule alone.  Fills min(n, strips) pairs (need may be NULL) and
 * returns the number of strips, or a negative lfc_status.  For tuning and
 * tests (lfc_decode_blocks_ex can cap the staging).
 */
int64_t lfc_stage_needs(const lfc_lf *lf, uint32_t *need, int64_t n);

/*
 * DecompressLFIBlock (Alg. 2) for a batch of blocks, decoded in parallel
 * (Sec. 3.6): each output block is the top key-view block plus the dequantised
 * residual blocks of its ancestors down to level 0 (Sec. 3.5), as int16 YCoCg-R
 * samples (Sec. 4), not clamped.
 *  d_req    device int32 [n][2] = {view index vi, block index b}, b row-major
 *           over the padded image's B x B blocks; or NULL for every block.
 *  n        number of requests; with d_req == NULL it must equal
 *           grid_u*grid_v*n_blocks (BLOCKS) or grid_u*grid_v (IMAGES).
 *           n == 0 with the BLOCKS layout does nothing (d_req may then be
 *           NULL, as an empty tensor's pointer is).
 *  layout   LFC_LAYOUT_BLOCKS: d_out is int16 [n][3][B][B], request order
 *           (d_req == NULL: order vi-major then b).
 *           LFC_LAYOUT_IMAGES (requires d_req == NULL): d_out is int16
 *           [grid_u*grid_v][3][padded_height][padded_width].
 * A request with vi or b out of range yields zeros and raises the handle's
 * device error flag, reported by lfc_check.  Errors: LFC_E_INVALID,
 * LFC_E_UNSUPPORTED (whole-field decode of a tree too large for on-chip
 * tables), LFC_E_HIP.
 */
lfc_status lfc_decode_blocks(const lfc_lf *lf, const int32_t *d_req, int64_t n, int32_t layout,
                             int16_t *d_out, hipStream_t s);

/*
 * lfc_decode_blocks with explicit launch settings (cfg NULL: automatic).
 *  stage_cap_words  LFC_LAYOUT_IMAGES only: at most this many 32-bit words
 *                   of LDS per workgroup for staging a strip's groups and
 *                   decode schedule (a strip whose need exceeds it reads them
 *                   from global memory; 0: no staging); -1: as the strips
 *                   need, within the workgroup's LDS budget.  Without a
 *                   config the handle's setting applies: no staging after
 *                   lfc_open, the measured choice after lfc_tune_decode.
 *                   Decoded samples do not depend on it.
 * Errors: as lfc_decode_blocks, plus LFC_E_INVALID (stage_cap_words < -1).
 */
typedef struct {
  int64_t stage_cap_words;
} lfc_decode_config;
lfc_status lfc_decode_blocks_ex(const lfc_lf *lf, const int32_t *d_req, int64_t n, int32_t layout,
                                int16_t *d_out, const lfc_decode_config *cfg, hipStream_t s);

/*
 * Measured tuning of the whole-field decode (LFC_LAYOUT_IMAGES): the
 * kernel decodes each strip's residual blocks in chunks that fit a tile of
 * stored blocks in LDS; a larger tile means fewer chunks but less LDS for
 * other uses.  The kernel can also copy each strip's groups and decode
 * schedule into LDS before decoding it (staging) or read them from global
 * memory.  This call times the decode (one warm-up, then `reps` launches,
 * events on stream s, output to d_out: int16, as the images layout) with the
 * handle's current tile capacity and with 3/4, 5/4, 6/4 and 7/4 of the
 * default (those that fit), each with and without staging, rebuilding the
 * strip tables for each capacity, and keeps the fastest pair in the handle
 * (lfc_decode_blocks without a config then uses it); res reports what was
 * tried.  Blocks until done.  The handle must not be in use by another call
 * meanwhile.  Decoded samples do not depend on the choice.
 * Errors: LFC_E_INVALID (null pointer, reps outside 1..1000, handle of
 * another device), LFC_E_NOMEM, LFC_E_HIP; on error the handle keeps the
 * tables and the staging it had.
 */
#define LFC_TUNE_DECODE_MAX 16
typedef struct {
  int32_t n_tried;
  int32_t best;                              /* index of the choice kept */
  int32_t tile_blocks[LFC_TUNE_DECODE_MAX];  /* stored blocks per tile */
  int32_t staged[LFC_TUNE_DECODE_MAX];       /* 1: strips staged in LDS, 0: read from global memory */
  float ms[LFC_TUNE_DECODE_MAX];             /* mean ms per decode */
} lfc_decode_tuning;
lfc_status lfc_tune_decode(lfc_lf *lf, int16_t *d_out, int32_t reps, lfc_decode_tuning *res, hipStream_t s);

/*
 * Progressive decompression (Sec. 3.6): the tree traversal of
 * DecompressLFIBlock (Alg. 2) stopped at tree level `level`, which yields the
 * filtered key-view value of the view's ancestor on that level: for each
 * (view, block) request, the key-view block plus the residual blocks of the
 * view's ancestors on levels L-2 down to `level`.  level 0 equals
 * lfc_decode_blocks; level L-1 is the key view alone.
 *  d_req, n, d_out  as lfc_decode_blocks with LFC_LAYOUT_BLOCKS.
 *  level            0..levels-1.
 * Out-of-range requests yield zeros and raise the device error flag.
 * Errors: LFC_E_INVALID, LFC_E_HIP.
 */
lfc_status lfc_decode_progressive(const lfc_lf *lf, const int32_t *d_req, int64_t n, int32_t level,
                                  int16_t *d_out, hipStream_t s);

/*
 * Every view decoded (Alg. 2 over all blocks, Sec. 3.5) and converted back to
 * 8-bit RGB (inverse YCoCg-R, each channel clamped to 0..255; Sec. 4): the
 * form a viewer or the decode-then-interpolate render consumes.
 *  d_out  device uint32 [grid_u*grid_v][padded_height][padded_width], 16-byte
 *         aligned; pixel = R | G << 8 | B << 16 (top byte zero).  Pixels of
 *         the padding hold the conversion of the padded samples.
 * Enqueued on s.  Errors: LFC_E_INVALID (null or too small buffer),
 * LFC_E_UNSUPPORTED (more than 2^32 pixels, or a tree whose tables exceed
 * the kernel's on-chip budget), LFC_E_HIP.
 */
lfc_status lfc_decode_rgb(const lfc_lf *lf, uint32_t *d_out, hipStream_t s);

/*
 * Measured choice of the colour whole-field kernel's tile capacity (the
 * kernel behind lfc_decode_rgb, the decode-then-interpolate renders and the
 * dense light fields of lfc_batch_render): times lfc_decode_rgb of every view
 * (one warm-up, then `reps` launches, events on stream s, output to d_out as
 * lfc_decode_rgb) with the handle's current capacity and with 4/8, 5/8, 6/8,
 * 7/8 and 10/8 of the default (those whose tile fits the LDS), rebuilding the
 * colour strip tables for each, and keeps the fastest in the handle unless it
 * is within 2 % of the current one (then the current stays); res reports
 * the capacities tried (staged[] all 0).  A smaller tile leaves room
 * for more workgroups per compute unit, a larger one needs fewer chunks per
 * strip; which wins depends on the light field.  Blocks until done.  The
 * handle must not be in use by another call (renders, batches) meanwhile.
 * Decoded and rendered results do not depend on the choice.
 * Errors: LFC_E_INVALID (null pointer, reps outside 1..1000, handle of
 * another device), LFC_E_UNSUPPORTED (a tree of one level), LFC_E_NOMEM,
 * LFC_E_HIP; on error the handle keeps the tables it had.
 */
lfc_status lfc_tune_decode_rgb(lfc_lf *lf, uint32_t *d_out, int32_t reps, lfc_decode_tuning *res, hipStream_t s);

/*
 * Novel-view rendering (Sec. 3.6): every output pixel is the quadrilinear
 * interpolation, over the two nearest camera columns, the two nearest
 * camera rows and the 2 x 2 nearest source pixels, of decoded samples
 * converted to RGB (inverse YCoCg-R, clamped to 0..255).  Source pixel
 * coordinates of output pixel (X, Y) are s + (X+0.5)*width/out_w - 0.5 and
 * t + (Y+0.5)*height/out_h - 0.5, clamped to the image.  The blocks under
 * each output tile are decoded on the fly, or, for large batches, the
 * source views the batch reads are decoded once (as 8-bit RGB) and the
 * pixels interpolated from them; both give the same bytes.  The decoded
 * views go to stream-ordered device scratch (4 x views x padded pixels
 * bytes) from a memory pool of the library's own per device, which keeps up
 * to 1 GiB of freed scratch for later calls until the process ends.
 *  d_views  device lfc_view [n].
 *  d_out    device float32 [n][3][out_h][out_w], RGB / 255.
 * Errors: LFC_E_INVALID (null pointer, n < 0, out_w or out_h < 1 or
 * > 16384), LFC_E_NOMEM (scratch), LFC_E_HIP.
 */
lfc_status lfc_render_views(const lfc_lf *lf, const lfc_view *d_views, int32_t n, int32_t out_w,
                            int32_t out_h, float *d_out, hipStream_t s);

/*
 * Launch shape of a render (results are the same bytes for every shape).
 *  LFC_RENDER_AUTO     the library's choice (decode-then-interpolate when the
 *                      batch's pixels are at least 1/20 of the light field's
 *                      samples, else tiles of up to 64 x 16 pixels).
 *  LFC_RENDER_TILES    one workgroup per output tile of tile_w x tile_h
 *                      pixels decodes the tile's source footprint (0 x 0:
 *                      64 x 16, shrunk until the footprint fits 64 KB).
 *  LFC_RENDER_DECODED  decode every source view, then interpolate.
 * disparity refocuses the render (the dynamic reparameterisation the paper
 * names as compatible with its decoder, Sec. 3.6): a novel camera at grid
 * position (u, v), clamped to the grid, samples source camera (iu, jv) at
 * image-plane offset (s + d (iu - u), t + d (jv - v)), so that a scene
 * plane whose image moves by -d pixels per camera step is in focus; d = 0 is
 * the plain two-plane interpolation of lfc_render_views.
 */
enum { LFC_RENDER_AUTO = 0, LFC_RENDER_TILES = 1, LFC_RENDER_DECODED = 2 };
typedef struct {
  int32_t path;
  int32_t tile_w, tile_h;   /* LFC_RENDER_TILES only, 1..1024 each, or both 0 */
  float disparity;          /* focal disparity d, finite, |d| <= 1e6 (0: none) */
} lfc_render_config;

/* lfc_render_views with an explicit launch shape and focal disparity (cfg
 * NULL: automatic, d = 0).  Errors: as lfc_render_views, plus LFC_E_INVALID
 * (unknown path, tile size, disparity) and LFC_E_UNSUPPORTED (the tile's
 * source footprint exceeds 64 KB). */
lfc_status lfc_render_views_ex(const lfc_lf *lf, const lfc_view *d_views, int32_t n, int32_t out_w,
                               int32_t out_h, float *d_out, const lfc_render_config *cfg, hipStream_t s);

/*
 * lfc_render_views_ex for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops, harnesses that forbid hipMalloc):
 * no allocation of any kind.  The decode-then-interpolate path decodes the
 * source views into a static device array of LFC_NOALLOC_SCRATCH_BYTES
 * (32 MiB), one per device, held from the first call on that device until
 * the process ends; the tile path needs no scratch.  Results are the bytes
 * lfc_render_views_ex gives for the same arguments.
 *  cfg  as lfc_render_views_ex.  The automatic choice takes the decoded path
 *       only when the light field's decoded views fit the scratch, else
 *       tiles; an explicit LFC_RENDER_DECODED whose decoded views do not fit
 *       fails with LFC_E_RANGE.
 * Every decoded-path call on one device shares that device's array, and
 * each call overwrites all of the part it reads before reading it: calls
 * that overlap in time on one device (different streams or threads) race,
 * so run them on one stream.
 * Errors: as lfc_render_views_ex, plus LFC_E_RANGE (decoded views larger
 * than the scratch), LFC_E_UNSUPPORTED (the automatic choice fell back to
 * tiles and the tile footprint does not fit), LFC_E_HIP (the scratch's
 * address cannot be found).
 */
#define LFC_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
lfc_status lfc_render_views_noalloc(const lfc_lf *lf, const lfc_view *d_views, int32_t n, int32_t out_w,
                                    int32_t out_h, float *d_out, const lfc_render_config *cfg, hipStream_t s);

/*
 * Measured tuning of the render's launch shape for one (light field, batch
 * size, output size): the decoded path and each tile shape of 32 x 8 up to
 * 256 x 8 pixels whose footprint fits are run once, then timed over `reps`
 * launches with events on stream s, on the caller's views (the output is
 * overwritten).  Blocks until the timing is done.  res->cfg[res->best] is
 * the fastest.  Allocates (and frees) the decoded path's scratch; when that
 * fails only tile shapes are tried.
 * Errors: as lfc_render_views, plus LFC_E_INVALID (n < 1, reps outside
 * 1..1000, null res), LFC_E_UNSUPPORTED (no shape fits).
 */
#define LFC_TUNE_MAX 16
typedef struct {
  int32_t n_tried;
  int32_t best;                          /* index of the fastest */
  lfc_render_config cfg[LFC_TUNE_MAX];
  float ms[LFC_TUNE_MAX];                /* mean ms per launch */
} lfc_render_tuning;
lfc_status lfc_render_tune(const lfc_lf *lf, const lfc_view *d_views, int32_t n, int32_t out_w, int32_t out_h,
                           float *d_out, int32_t reps, lfc_render_tuning *res, hipStream_t s);

/*
 * A render plan: one render of n views at out_w x out_h with its launch
 * shape fixed (cfg, NULL: automatic), its device pointers fixed, and, with
 * graph != 0, its launches captured once into a HIP graph, so that each
 * lfc_render_plan_launch is one graph launch.  The views are read at each
 * launch, so the caller may rewrite d_views between launches.  The decoded
 * path's scratch (the light field's decoded views) is allocated at creation
 * and held by the plan.  Launches of one plan must not overlap (use one
 * stream); the light field and both buffers must outlive the plan.
 * lfc_render_plan_destroy waits for the device (it frees device memory).
 * lfc_render_plan_info reports the resolved shape and whether a graph is used.
 * Errors: as lfc_render_views_ex, plus LFC_E_NOMEM (scratch), LFC_E_HIP
 * (capture or instantiation).
 */
typedef struct lfc_render_plan lfc_render_plan;
lfc_status lfc_render_plan_create(const lfc_lf *lf, const lfc_render_config *cfg, const lfc_view *d_views,
                                  int32_t n, int32_t out_w, int32_t out_h, float *d_out, int32_t graph,
                                  lfc_render_plan **plan);
lfc_status lfc_render_plan_launch(lfc_render_plan *plan, hipStream_t s);
lfc_status lfc_render_plan_info(const lfc_render_plan *plan, lfc_render_config *cfg, int32_t *graph);
void lfc_render_plan_destroy(lfc_render_plan *plan);

/*
 * Batched rendering across light fields.  Views are independent of each
 * other (any block of any view decodes on its own, Sec. 3.5, and a view is
 * rendered from the blocks under its footprint, Sec. 3.6), so requests for
 * several light fields and output sizes share one launch per block size in
 * use.  Each result is bit-identical to lfc_render_views of that request
 * alone.
 */
typedef struct {
  int32_t lf;               /* index into the lfs array of the call */
  int32_t out_w, out_h;     /* output size, 1..16384 each */
  lfc_view view;            /* camera and image-plane offset, as lfc_render_views */
} lfc_render_request;

typedef struct lfc_batch lfc_batch;   /* staging for request tables; opaque */

/* A batch context for the current device.  Errors: LFC_E_INVALID, LFC_E_NOMEM, LFC_E_HIP. */
lfc_status lfc_batch_create(lfc_batch **out);

/*
 *  lfs     host array of n_lf open handles, all on the current device.
 *  reqs    host array of n requests (n >= 0); reqs[i].lf indexes lfs.
 *  d_outs  host array of n device pointers, 4-byte aligned; d_outs[i]
 *          receives float32 [3][out_h][out_w], RGB / 255.
 * The request table is packed on the host and copied to the device on s.
 * The context keeps four tables: four calls may be in flight, on any
 * streams, and a fifth waits until the kernels of the first have finished
 * (a table is never rewritten while a launch may still read it).  The
 * staging grows on demand (a call with more requests than any before
 * allocates).
 * Paths (Sec. 3.6: decode the blocks a view needs, then interpolate): a
 * light field whose requests in the call cover at least a twentieth of the
 * pixels it holds is decoded once, only the views its requests read, as
 * 8-bit RGB, by one persistent launch over every such light field of a block
 * size (workgroups take (strip, part) items of all of them from a device
 * counter), then one launch interpolates all those requests; the other
 * requests render by output tiles, each decoding its footprint.  Both give
 * the bytes lfc_render_views gives for the request alone.  The decoded views
 * live in device buffers the context allocates on first use per light field
 * (4 x views x padded pixels bytes) and keeps until it is destroyed; a
 * light field for which no buffer can be allocated renders by tiles.
 * Errors:
 * LFC_E_INVALID (null pointer, index or size out of range, more than 65535
 * requests of one block size), LFC_E_UNSUPPORTED, LFC_E_NOMEM, LFC_E_HIP.
 */
lfc_status lfc_batch_render(lfc_batch *b, const lfc_lf *const *lfs, int32_t n_lf, const lfc_render_request *reqs,
                            int32_t n, float *const *d_outs, hipStream_t s);

/*
 * Random access (DecompressLFIBlock, Alg. 2) over several light fields in one
 * launch: request i = d_req[3i..3i+2] = (index into lfs, view, block), every
 * light field of the call with the same block size B.  d_out is int16
 * [n][3][B][B] (16-byte aligned), as lfc_decode_blocks with LFC_LAYOUT_BLOCKS.
 * Out-of-range requests yield zeros and raise the batch's error flag, read by
 * lfc_batch_check.  The light-field table shares the request-table staging
 * of lfc_batch_render.  Errors: LFC_E_INVALID, LFC_E_UNSUPPORTED (mixed block
 * sizes), LFC_E_NOMEM, LFC_E_HIP.
 */
lfc_status lfc_batch_decode(lfc_batch *b, const lfc_lf *const *lfs, int32_t n_lf, const int32_t *d_req, int64_t n,
                            int16_t *d_out, hipStream_t s);

/* Waits for stream s, then reads and clears the batch's error flag
 * (LFC_E_INVALID if a batched decode saw an out-of-range request). */
lfc_status lfc_batch_check(lfc_batch *b, hipStream_t s);

/* Waits for the context's work and frees it.  NULL is ignored. */
lfc_status lfc_batch_destroy(lfc_batch *b);

/*
 * A batch plan: one lfc_batch_render call fixed once (the same light fields,
 * requests and output pointers at every launch), with its request table
 * copied to the device at creation, its decoded-view buffers allocated then
 * and held by the plan, and, with graph != 0, its launches captured once
 * into a HIP graph, so that each lfc_batch_plan_launch is one graph launch
 * (the graph holds kernels only; the persistent colour decode leaves its
 * work counters at zero for the next launch).  Each launch writes what
 * lfc_batch_render of the same arguments writes.  Launches of one plan must
 * not overlap (use one stream); the light fields and the output buffers
 * must outlive the plan.  lfc_batch_plan_destroy waits for the device (it
 * frees device memory); NULL is ignored.  lfc_batch_plan_info reports how
 * many light fields take the decoded colour path and whether a graph is
 * used.  Errors: as lfc_batch_render (n must be at least 1), plus LFC_E_HIP
 * (capture or instantiation).
 */
typedef struct lfc_batch_plan lfc_batch_plan;
lfc_status lfc_batch_plan_create(const lfc_lf *const *lfs, int32_t n_lf, const lfc_render_request *reqs, int32_t n,
                                 float *const *d_outs, int32_t graph, lfc_batch_plan **plan);
lfc_status lfc_batch_plan_launch(lfc_batch_plan *plan, hipStream_t s);
lfc_status lfc_batch_plan_info(const lfc_batch_plan *plan, int32_t *n_decoded_lf, int32_t *graph);
void lfc_batch_plan_destroy(lfc_batch_plan *plan);

/*
 * Serving loop over resident light fields (the access pattern the paper
 * designs for: many novel views of compressed light fields kept in GPU
 * memory, Sec. 1 and 3.5).  Requests are queued on submit; one engine thread
 * launches every queued request it can admit as one batch whenever one of
 * `streams` launch slots is free (continuous batching), up to max_batch per
 * launch.  Results live in a device pool of out_pool_bytes; a request whose
 * output does not fit waits, in arrival order, until released results make
 * room (memory admission).  max_batch = 1 with one stream is one plain
 * launch per request.
 */
typedef struct lfc_server lfc_server;

typedef struct {
  int32_t max_batch;        /* requests per launch, 1..65535 */
  int32_t streams;          /* launches in flight, 1..8; each on a stream of its own */
  int64_t out_pool_bytes;   /* device bytes for results, >= 256 */
  int64_t max_queue;        /* requests waiting for admission at most (0: no limit); a submit
                               beyond it is refused with LFC_E_NOMEM */
  int64_t device_bytes_cap; /* device memory the server may count on (0: no cap): the resident
                               light fields (lfc_info device_bytes) plus the output pool must fit
                               (else lfc_server_create refuses with LFC_E_NOMEM); the decoded-view
                               buffers of the batches' colour path (one per light field and
                               stream) are granted from what remains, light field by light field
                               in order, and a light field without one renders by tiles */
} lfc_server_config;

typedef struct {
  int64_t submitted, completed, batches;
  int64_t max_batch_seen;   /* most requests in one launch */
  int64_t admission_waits;  /* times the head of the queue waited for pool room */
  int64_t pool_bytes_in_use;
} lfc_server_stats;

/* Copies the lfs array (the handles must outlive the server).  Errors:
 * LFC_E_INVALID, LFC_E_NOMEM (no host memory, no output pool, or the light
 * fields and pool exceed device_bytes_cap), LFC_E_HIP. */
lfc_status lfc_server_create(const lfc_lf *const *lfs, int32_t n_lf, const lfc_server_config *cfg,
                             lfc_server **out);

/* Queues one request; *ticket identifies it.  Thread-safe.  Errors:
 * LFC_E_INVALID (bad index or size, or an output larger than the pool),
 * LFC_E_NOMEM (max_queue requests already wait for admission). */
lfc_status lfc_server_submit(lfc_server *sv, const lfc_render_request *req, uint64_t *ticket);

/* Blocks until the request is done (timeout_ms < 0: no limit); *d_img is
 * then its result in the pool (device float32 [3][out_h][out_w]) and
 * *latency_ms the time from submit to completion.  The result stays valid
 * until lfc_server_release.  Errors: LFC_E_INVALID (unknown ticket, or the
 * timeout passed), the launch's status if it failed. */
lfc_status lfc_server_wait(lfc_server *sv, uint64_t ticket, int32_t timeout_ms, const float **d_img,
                           double *latency_ms);

/* Returns the request's result memory to the pool and forgets the ticket.
 * The memory may be handed to the next request at once: every read of the
 * result (a copy included) must have completed before this call. */
lfc_status lfc_server_release(lfc_server *sv, uint64_t ticket);

/* Submits reqs[i] at arrival_ms[i] after the call starts (non-decreasing
 * times), results discarded on completion, and returns once all are done
 * with latency_ms[i] (host array of n) from each arrival to completion;
 * a request refused because the queue was full gets latency -1. */
lfc_status lfc_server_replay(lfc_server *sv, const lfc_render_request *reqs, const double *arrival_ms, int32_t n,
                             double *latency_ms);

lfc_status lfc_server_get_stats(lfc_server *sv, lfc_server_stats *st);

/* Stops the engine after the queued work, waits for it and frees the
 * server.  NULL is ignored. */
lfc_status lfc_server_destroy(lfc_server *sv);

/*
 * Waits for stream s, then reads and clears the handle's device error flag.
 * Returns LFC_E_INVALID if a decode since the last check saw an
 * out-of-range request, LFC_E_HIP on a runtime error, else LFC_OK.
 */
lfc_status lfc_check(const lfc_lf *lf, hipStream_t s);

/* Frees the handle and its device memory.  Work using it must have
 * completed.  NULL is ignored. */
lfc_status lfc_close(lfc_lf *lf);

/* Message for the last non-OK status returned on this thread. */
const char *lfc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif

// Internal declarations shared by the host side (host.cpp), the HIP kernels
// (kernels.hip, mlp.hip) and the runtime (serve.cpp) of liblfc.so.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/lfc.h"

namespace lfc {

constexpr int kMaxLevels = LFC_MAX_LEVELS;
constexpr int kNumCodes = 26;           // BISE range codes 0..25
constexpr uint32_t kAllCodes = (1u << kNumCodes) - 1u;
constexpr int kHeaderBytes = 128;

// Geometry derived from the parameters (grid sizes per tree level, padded
// image, blocks, groups).
struct Geometry {
  int U = 0, V = 0, W = 0, H = 0, B = 0, S = 0, L = 0, q = 0;
  int wp = 0, hp = 0, nbx = 0, nby = 0, nb = 0, ng = 0;
  int n_srv = 0, n_top = 0, nbw = 0;    // nbw: bitmap words per group
  int lu[kMaxLevels] = {0}, lv[kMaxLevels] = {0}, c[kMaxLevels] = {0};
  int nv() const { return U * V; }
};

// Fills g from p; returns LFC_OK or LFC_E_INVALID with the reason in *why.
lfc_status make_geometry(const lfc_params &p, Geometry &g, std::string *why);

// Tree tables.  path[vi*(L-1) + l] is the serial (BFS) index of the level-l
// ancestor of view vi, root[vi] the top-level node.  batch holds the views in
// the serial order of level 0, cut into runs of at most kBatch siblings (views
// with the same ancestors), one kBatchWords-word record per run:
//   [0] n, [1..4] view indices (-1 unused), [5] root, [6..9] serial indices of
//   the ancestors from level L-2 down to level 1 (-1 unused), [10] serial
//   index of the first view of the run (the others follow it), [11..15] unused.
constexpr int kBatch = 4;
constexpr int kBatchWords = 16;
// Default capacity, in stored residual blocks, of the whole-field kernel's
// compact tile (32 KB of LDS; tile slots are 11-bit, beside a 5-bit block
// index in 16-bit schedule items, so at most 2048).
constexpr int tile_blocks(int B) { return B == 2 ? 2048 : (B == 4 ? 1024 : 256); }
// Words per entry of the whole-field kernel's strip order: the strip, its
// decode schedule's first word and length, a spare word, then its 64/B
// groups' start words and lengths (zero past the image's right edge), so a
// workgroup reads everything it needs to start a strip in one load.
constexpr int order_words(int B) { return 4 + 2 * (64 / B); }
// Most words of a chunk's gather table (per-node masks and first slots,
// per-run node positions) in the whole-field kernel's schedule: the kernel
// copies a chunk's table into LDS when the strip is read from global memory.
constexpr int kLFTabWords = 1024;
// Most tree nodes in one chunk of the colour whole-field kernel's schedule
// (the kernel copies a chunk's per-node tables into LDS).
constexpr int kRGBNodeCap = 128;
struct TreeTables {
  std::vector<int32_t> path, root, batch;
  std::vector<std::vector<int32_t>> serial;  // [level][node id] -> BFS index (-1 on top)
};
void build_tree_tables(const Geometry &g, TreeTables &t);

// Bits of a BISE block of S values under range code k.
int bise_block_bits(int code, int S);
// Control rows of a geometry: every residual (node, block, channel).
int64_t control_rows(const Geometry &g);
// The encoder's per-block network on the GPU: n feature rows (host) to the
// threshold class, range class and top threshold-class probability (host).
lfc_status mlp_infer_rows(const void *d_w, const float *feat, int64_t n, int8_t *cls, int8_t *rng, float *conf,
                          hipStream_t s);

// Records a failure for lfc_last_error and returns st.
lfc_status fail(lfc_status st, const std::string &msg);

}  // namespace lfc

// Device-resident compressed light field.
struct lfc_lf {
  lfc_params params;
  lfc::Geometry geo;
  int device = 0;
  uint64_t stream_bytes = 0, present = 0;
  void *d_base = nullptr;      // one allocation holding everything below
  size_t d_bytes = 0;
  const int16_t *d_rkv = nullptr;    // [n_top][nb][3][S]
  const uint32_t *d_off = nullptr;   // [ng+1] group start words
  const uint32_t *d_srv = nullptr;   // SRV words, zero-padded at the end
  const uint32_t *d_dbase = nullptr; // [ng][nbw] directory index of each bitmap word's first node
  const uint32_t *d_poff = nullptr;  // [present] (payload bit offset in group << 5) | code
  const uint32_t *d_pbase = nullptr; // [ng+1] index in d_poff of each group's first stored block
  const uint32_t *d_dir2 = nullptr;  // [nb][nbw][3][2] per block, bitmap word and channel: (bitmap word, d_dbase entry)
  const int32_t *d_path = nullptr;   // [nv][L-1]
  const int32_t *d_root = nullptr;   // [nv]
  const int32_t *d_batch = nullptr;  // [n_batch][kBatchWords]
  int n_batch = 0;
  const uint32_t *d_sched = nullptr;     // decode schedule of the whole-field kernel (strip records)
  const uint32_t *d_strip_off = nullptr; // [n_strips+1] word offset of each strip's record
  const uint32_t *d_order = nullptr;     // [n_strips] strips in the order the whole-field kernel takes them
  const uint32_t *d_sched_rgb = nullptr;     // colour decode schedule (strips of all three channels)
  const uint32_t *d_strip_off_rgb = nullptr; // [n_strips_rgb+1]
  const uint32_t *d_order_rgb = nullptr;     // [n_strips_rgb] costliest first
  int tile_cap_rgb = 0;              // blocks of the colour kernel's compact tile
  int rgb_max_chunks = 1;            // most chunks of one strip in the colour schedule
  int32_t *d_err = nullptr;          // device error flag
  int tile_cap = 0;                  // blocks of the whole-field kernel's compact residual tile
  int64_t stage_cap = 0;             // LDS words for staging a strip (-1: as it needs, 0: none); the
                                     // setting used when a decode call gives none
  void *d_sched_own = nullptr;       // strip tables chosen by lfc_tune_decode (else inside d_base)
  void *d_sched_rgb_own = nullptr;   // colour strip tables chosen by lfc_tune_decode_rgb (else inside d_base)
  uint32_t max_strip_words = 0;      // largest group words + decode schedule of a strip of 64/B blocks of
                                     // one channel
  std::vector<uint32_t> strip_need;  // per strip: group words + schedule words, schedule words
};

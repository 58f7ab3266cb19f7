// Host-code driver for the sanitizer build (AddressSanitizer and
// UndefinedBehaviorSanitizer, no GPU needed): the oracle (plain C) and the
// library's host code (encoder, stream validator, decoder initialisation
// with its directory and strip-table builders) run over synthetic light
// fields of several geometries, then the validator and the initialisation
// over corrupted copies of each stream (bit flips, truncations).
//
// The library's GPU entry points that host.cpp calls are replaced by stubs
// here; lfc_open stops at the device allocation on a machine without a GPU
// (after every host table is built) and returns LFC_E_HIP.
//
// Exit status 0 when every check holds; a sanitizer report aborts the run.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../include/lfc.h"
extern "C" {
#include "../oracle/oracle.h"
}

// stubs for the GPU calls of host.cpp (never reached without a device)
namespace lfc {
lfc_status mlp_infer_rows(const void *, const float *, int64_t, int8_t *, int8_t *, float *, hipStream_t) {
  return LFC_E_UNSUPPORTED;
}
}  // namespace lfc
extern "C" lfc_status lfc_decode_blocks(const lfc_lf *, const int32_t *, int64_t, int32_t, int16_t *, hipStream_t) {
  return LFC_E_UNSUPPORTED;
}
extern "C" lfc_status lfc_decode_rgb(const lfc_lf *, uint32_t *, hipStream_t) { return LFC_E_UNSUPPORTED; }

namespace {

int failures = 0;

void check(bool ok, const char *what, int geom) {
  if (!ok) {
    std::fprintf(stderr, "FAIL geometry %d: %s\n", geom, what);
    failures++;
  }
}

uint64_t splitmix(uint64_t &s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// smooth gradients shifted per view (a little parallax) plus noise
std::vector<uint8_t> light_field(int U, int V, int W, int H, uint64_t seed) {
  std::vector<uint8_t> rgb((size_t)U * V * W * H * 3);
  uint64_t s = seed;
  for (int v = 0; v < V; v++)
    for (int u = 0; u < U; u++)
      for (int y = 0; y < H; y++)
        for (int x = 0; x < W; x++)
          for (int c = 0; c < 3; c++) {
            const int base = (x + 2 * u) * (3 + c) + (y + v) * (5 - c) + 40 * c;
            const int noise = (int)(splitmix(s) % 9) - 4;
            int val = base % 256 + noise;
            val = val < 0 ? 0 : (val > 255 ? 255 : val);
            rgb[((((size_t)v * U + u) * H + y) * W + x) * 3 + c] = (uint8_t)val;
          }
  return rgb;
}

struct Geom {
  int U, V, W, H, B, L, c[5], tpix, tblk, q;
  uint32_t mask;
};

const Geom kGeoms[] = {
    {8, 8, 64, 64, 4, 2, {2}, 0, 2, 0, 0},
    {1, 1, 12, 10, 4, 1, {0}, 0, 0, 0, 0},
    {3, 5, 13, 9, 4, 2, {2}, 0, 0, 0, 0},
    {17, 17, 20, 12, 4, 3, {2, 3}, 0, 30, 1, 0},
    {9, 9, 70, 43, 4, 3, {2, 2}, 2, 20, 2, 0},
    {5, 4, 72, 24, 8, 2, {3}, 0, 60, 3, 0},
    {6, 3, 130, 10, 2, 3, {2, 2}, 1, 3, 0, 0},
    {7, 7, 33, 17, 4, 4, {2, 2, 2}, 0, 10, 4, 0},
    {4, 4, 150, 8, 4, 2, {2}, 0, 0, 0, 0x3F80000u | 0x7F000u | (0xFu << 8)},
    {2, 3, 64, 64, 4, 6, {2, 2, 2, 2, 2}, 0, 0, 0, 0},
};

void run(int gi, const Geom &gm) {
  const std::vector<uint8_t> rgb = light_field(gm.U, gm.V, gm.W, gm.H, 1000 + gi);
  // the oracle: encode, decode every block, random access, a render
  orc_params op{};
  op.grid_u = gm.U;
  op.grid_v = gm.V;
  op.width = gm.W;
  op.height = gm.H;
  op.block = gm.B;
  op.levels = gm.L;
  for (int l = 0; l < gm.L - 1; l++) op.cluster[l] = gm.c[l];
  op.pix_threshold = gm.tpix;
  op.blk_threshold = gm.tblk;
  op.quant_bits = gm.q;
  op.range_mask = gm.mask;
  orc_geom og{};
  check(orc_geometry(&op, &og) == ORC_OK, "oracle geometry", gi);
  const size_t samples = (size_t)gm.U * gm.V * 3 * og.hp * og.wp;
  std::vector<int16_t> r0(samples), dec(samples);
  uint8_t *ostream = nullptr;
  int64_t obytes = 0;
  check(orc_encode(rgb.data(), &op, &ostream, &obytes, r0.data(), nullptr, nullptr) == ORC_OK, "oracle encode", gi);
  check(orc_decode_all(ostream, obytes, 0, og.nb, dec.data()) == ORC_OK, "oracle decode_all", gi);
  check(dec == r0, "oracle decode_all equals the closed-loop reconstruction", gi);
  int16_t blk[3 * 64];
  for (int k = 0; k < 16; k++) {
    const int vi = k % (gm.U * gm.V), b = (k * 7919) % og.nb;
    check(orc_decode_block(ostream, obytes, vi, b, blk) == ORC_OK, "oracle decode_block", gi);
  }
  const float views[8] = {0.5f * (gm.U - 1), 0.25f * (gm.V - 1), 0.5f, -0.5f, (float)gm.U, -1.0f, 2.0f, 1.0f};
  std::vector<float> img(2 * 3 * 17 * 13);
  check(orc_render(r0.data(), gm.U, gm.V, gm.W, gm.H, og.wp, og.hp, views, 2, 17, 13, img.data()) == ORC_OK,
        "oracle render", gi);

  // the library's host encoder: the same stream as the oracle's
  lfc_params lp{};
  lp.grid_u = gm.U;
  lp.grid_v = gm.V;
  lp.width = gm.W;
  lp.height = gm.H;
  lp.block = gm.B;
  lp.levels = gm.L;
  for (int l = 0; l < gm.L - 1; l++) lp.cluster[l] = gm.c[l];
  lp.pix_threshold = gm.tpix;
  lp.blk_threshold = gm.tblk;
  lp.quant_bits = gm.q;
  lp.range_mask = gm.mask;
  void *lstream = nullptr;
  size_t lbytes = 0;
  check(lfc_encode(rgb.data(), &lp, &lstream, &lbytes) == LFC_OK, "library encode", gi);
  check(lbytes == (size_t)obytes && std::memcmp(lstream, ostream, lbytes) == 0, "library stream equals the oracle's",
        gi);
  lfc_params back{};
  check(lfc_validate(lstream, lbytes, &back) == LFC_OK, "validate", gi);
  // initialisation: every host table is built; without a GPU the device
  // allocation then fails
  lfc_lf *lf = nullptr;
  lfc_status st = lfc_open(lstream, lbytes, nullptr, &lf);
  check(st == LFC_OK || st == LFC_E_HIP, "open", gi);
  if (lf) lfc_close(lf);

  // corrupted copies: flipped bits and truncations never crash the validator
  // or the initialisation
  std::vector<uint8_t> bad(static_cast<uint8_t *>(lstream), static_cast<uint8_t *>(lstream) + lbytes);
  uint64_t s = 77 + gi;
  const int flips = 160;
  for (int k = 0; k < flips; k++) {
    // the header and the offsets section first, then anywhere
    const size_t limit = k < flips / 2 ? std::min<size_t>(lbytes, 4096) : lbytes;
    const size_t at = (size_t)(splitmix(s) % limit);
    const uint8_t bit = (uint8_t)(1u << (splitmix(s) % 8));
    bad[at] ^= bit;
    lfc_params pp{};
    if (lfc_validate(bad.data(), bad.size(), &pp) == LFC_OK) {
      lfc_lf *h = nullptr;
      const lfc_status so = lfc_open(bad.data(), bad.size(), nullptr, &h);
      check(so == LFC_OK || so == LFC_E_HIP, "open of a stream that validates", gi);
      if (h) lfc_close(h);
    } else {
      lfc_lf *h = nullptr;
      check(lfc_open(bad.data(), bad.size(), nullptr, &h) != LFC_OK && !h, "open refuses what validate refuses", gi);
    }
    bad[at] ^= bit;
  }
  for (int k = 0; k < 48; k++) {
    const size_t len = k < 24 ? (size_t)k * 7 : (size_t)(splitmix(s) % lbytes);
    lfc_params pp{};
    check(lfc_validate(bad.data(), len, &pp) != LFC_OK, "truncated stream refused", gi);
  }
  lfc_free(lstream);
  orc_free(ostream);
}

}  // namespace

int main() {
  int gi = 0;
  for (const Geom &gm : kGeoms) run(gi++, gm);
  std::printf("%d geometries, %d failures\n", gi, failures);
  return failures ? 1 : 0;
}

// HIP kernels for gfx950 (CDNA4, wave64) and the exported calls that launch
// them: decoding (lfc_decode_blocks, lfc_decode_progressive), rendering
// (lfc_render_views, lfc_render_views_ex, lfc_render_tune, the render
// plans), and the launchers the batch context and server use.
//
// Decoding a block (Alg. 2, Sec. 3.5) is: read the top-level key-view block,
// then for every level below, locate the node's residual block inside the
// group of its spatial location (one level of indirection through the
// block offsets, Sec. 3.4), unpack its BISE values (Sec. 3.3), undo the
// zigzag and the quantiser step, and add it.  All integer work; no MFMA.
//
// Work mapping of the whole-field kernel: a workgroup owns a strip of 64/B
// blocks of one block row and channel; one lane decodes a whole stored
// residual block into LDS, then each lane gathers and stores 16 bytes of an
// output row (key view + ancestors + leaf).  Random access and rendering
// give one lane one row of B samples of a block.  Samples travel as packed
// int16 pairs: the residual tail (zigzag undo, step 2^q, adding the parent)
// runs on both halves of a register at once, and the sums wrap modulo 2^16
// exactly as the final int16 store of a 32-bit sum would.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "internal.h"
#include "serve.h"

// Device memory of lfc_render_views_noalloc: the decoded source views of
// its decode-then-interpolate path, for callers that cannot allocate.  Each
// device that runs the library holds its own copy until the process ends;
// host code reaches it only through the address hipGetSymbolAddress returns
// on that device.
static __device__ __align__(256) uint8_t scratch[LFC_NOALLOC_SCRATCH_BYTES];

namespace {

using lfc::kMaxLevels;
constexpr uint32_t kAbsent = 0xFFFFFFFFu;
constexpr int kLutEntries = 384;  // 256 trit-field values, then 128 quint-field values
constexpr int kThreads = 256;

// Range code k: 0..11 bits (m = k+1), 12..18 trits (m = k-12), 19..25 quints (m = k-19).
__device__ __forceinline__ uint32_t code_kind(uint32_t k) { return k < 12u ? 0u : (k < 19u ? 1u : 2u); }
__device__ __forceinline__ uint32_t code_m(uint32_t k) { return k < 12u ? k + 1u : (k < 19u ? k - 12u : k - 19u); }

template <int S>
struct Planes {
  static constexpr uint32_t trit = (8 * S + 4) / 5;    // digit-plane bits, trit blocks
  static constexpr uint32_t quint = (7 * S + 2) / 3;   // digit-plane bits, quint blocks
};

template <int S>
__device__ __forceinline__ uint32_t block_bits(uint32_t code) {
  const uint32_t kind = code_kind(code), m = code_m(code);
  return S * m + (kind == 0u ? 0u : (kind == 1u ? Planes<S>::trit : Planes<S>::quint));
}

// Digits of a trit field (entries 0..255: five 2-bit digits) or of a quint
// field (entries 256..383: three 3-bit digits).  Out-of-range fields map to 0;
// streams holding them are rejected before upload.
constexpr uint32_t lut_value(int t) {
  uint32_t v = 0;
  if (t < 256) {
    if (t < 243)
      for (int r = 0, x = t, p = 0; r < 5; r++, x /= 3, p += 2) v |= (uint32_t)(x % 3) << p;
  } else if (t - 256 < 125) {
    for (int r = 0, x = t - 256, p = 0; r < 3; r++, x /= 5, p += 3) v |= (uint32_t)(x % 5) << p;
  }
  return v;
}
__device__ __forceinline__ uint16_t lut_entry(int t) { return (uint16_t)lut_value(t); }

// The LUT, two entries per word, as a table in device memory (the
// whole-field kernel copies it into LDS instead of computing it).
struct LutWords {
  uint32_t w[kLutEntries / 2];
};
constexpr LutWords make_lut_words() {
  LutWords l{};
  for (int t = 0; t < kLutEntries; t++) l.w[t / 2] |= lut_value(t) << (16 * (t & 1));
  return l;
}
__device__ constexpr LutWords kLutTable = make_lut_words();

// 64 bits of a group's bit stream starting at bit pos (bit p is bit p%32 of word p/32).
__device__ __forceinline__ uint64_t window64(const uint32_t *gw, uint32_t pos) {
  const uint32_t *p = gw + (pos >> 5);
  const uint32_t a = p[0], b = p[1], c = p[2];
  const uint32_t sh = pos & 31u;
  const uint32_t lo = __builtin_amdgcn_alignbit(b, a, sh);
  const uint32_t hi = __builtin_amdgcn_alignbit(c, b, sh);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t join64(const uint32_t v[3], uint32_t sh) {
  return ((uint64_t)__builtin_amdgcn_alignbit(v[2], v[1], sh) << 32) | __builtin_amdgcn_alignbit(v[1], v[0], sh);
}

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ u16x2 as_u16x2(uint32_t v) { return __builtin_bit_cast(u16x2, v); }
__device__ __forceinline__ uint32_t as_u32(u16x2 v) { return __builtin_bit_cast(uint32_t, v); }

// two samples at once: a + b modulo 2^16 per half
__device__ __forceinline__ uint32_t add_pk(uint32_t a, uint32_t b) { return as_u32(as_u16x2(a) + as_u16x2(b)); }

// Two zigzagged values (0,1,2,3,.. -> 0,-1,1,-2,..) in the 16-bit halves of
// z, back to signed and times 2^q (0 <= q <= 4), as int16 pairs.  A value's
// magnitude times 2^q is (z >> 1) << q = z rotated left by q - 1 (right by
// 1 for q = 0) with the low half's top bit and the word's top bit cleared;
// a negative value's bits from q - 1 up are then inverted, which also clears
// bit q - 1 (its zigzag parity bit).  Every zigzag value of a valid stream is
// below 2^12 (at most 12 plain bits, or 6 bits below a trit or quint digit),
// so nothing crosses between the halves; equal, for all such pairs and every
// q, to unzigzagging each half and shifting it left by q (checked
// exhaustively on the host by tests/arith_identities.c).  Five VALU
// operations per pair against seven with packed 16-bit shifts.
__device__ __forceinline__ uint32_t unzigzag_pk(uint32_t z, int q) {
  const uint32_t rot = (uint32_t)(33 - q) & 31u;
  const uint32_t inv = q ? (0xFFFFu << (q - 1)) & 0xFFFFu : 0xFFFFu;   // the bits a negative value inverts
  const uint32_t t = __builtin_amdgcn_alignbit(z, z, rot) & 0x7FFF7FFFu;
  return t ^ ((z & 0x00010001u) * inv);
}

// Where the digits of row y (values y*B .. y*B+B-1) sit in a trit or quint
// block: bits 0..7 the bit offset of the row's first digit field in the
// digit plane, bits 8..15 the offset of the row's first digit in the
// concatenated digits of those fields, bits 16+4i the width of the row's i-th
// field (the last group of a block can be short; 0 = no such field).
// Computed once per lane.
template <int B>
__device__ __forceinline__ uint32_t digit_plan(int y, bool trit) {
  constexpr int S = B * B;
  const int glen = trit ? 5 : 3, fw = trit ? 8 : 7, dbits = trit ? 2 : 3;
  const int rem = S % glen, last = S / glen;
  const int pw = trit ? (8 * rem + 4) / 5 : (7 * rem + 2) / 3;
  const int i0 = y * B, a = i0 / glen, a_end = (i0 + B - 1) / glen;
  uint32_t plan = (uint32_t)(a * fw) | ((uint32_t)((i0 - a * glen) * dbits) << 8);
  for (int i = 0; i <= a_end - a && i < 4; i++)
    plan |= (uint32_t)((rem && a + i == last) ? pw : fw) << (16 + 4 * i);
  return plan;
}

// Words of one row's BISE fields, read before any of them is used so that the
// reads of several blocks can be in flight together.
template <int B>
struct RowWords {
  uint32_t l[3];     // low-bit plane from value i0
  uint32_t l2[3];    // low-bit plane from value i0+4 (B == 8)
  uint32_t dg[2];    // the row's digit fields
};

template <int B>
__device__ __forceinline__ void fetch_row(const uint32_t *gw, uint32_t e, uint32_t plan_t, uint32_t plan_q, int y,
                                          RowWords<B> &w) {
  constexpr int S = B * B;
  const uint32_t code = e & 31u, rel = e >> 5;
  const bool is_bits = code < 12u, is_trit = code - 12u < 7u;
  const uint32_t m = is_bits ? code + 1u : (is_trit ? code - 12u : code - 19u);
  const uint32_t hdr = is_bits ? 0u : (is_trit ? Planes<S>::trit : Planes<S>::quint);
  const uint32_t p = rel + hdr + (uint32_t)(y * B) * m;
  const uint32_t *q = gw + (p >> 5);
  w.l[0] = q[0];
  w.l[1] = q[1];
  w.l[2] = q[2];
  if constexpr (B > 4) {
    const uint32_t *q2 = gw + ((p + 4u * m) >> 5);
    w.l2[0] = q2[0];
    w.l2[1] = q2[1];
    w.l2[2] = q2[2];
  }
  const uint32_t pd = rel + (is_bits ? 0u : ((is_trit ? plan_t : plan_q) & 0xffu));
  const uint32_t *qd = gw + (pd >> 5);
  w.dg[0] = qd[0];
  w.dg[1] = qd[1];
}

// BISE unpack of the row (digit << m | low bits), zigzag undo, times 2^q:
// d holds the B residuals as B/2 packed int16 pairs.
template <int B>
__device__ __forceinline__ void finish_row(const RowWords<B> &w, uint32_t e, uint32_t plan_t, uint32_t plan_q, int y,
                                           int q, const uint16_t *lut, uint32_t d[B / 2]) {
  constexpr int S = B * B, NF = B == 8 ? 4 : 2;
  using DigitWord = std::conditional_t<B == 8, uint64_t, uint32_t>;
  const uint32_t code = e & 31u, rel = e >> 5;
  const bool is_bits = code < 12u, is_trit = code - 12u < 7u;
  const uint32_t m = is_bits ? code + 1u : (is_trit ? code - 12u : code - 19u);
  const uint32_t hdr = is_bits ? 0u : (is_trit ? Planes<S>::trit : Planes<S>::quint);
  const uint32_t p = rel + hdr + (uint32_t)(y * B) * m;
  const uint32_t lmask = (1u << m) - 1u;
  uint32_t low[B];
  {
    const uint64_t v = join64(w.l, p & 31u);
#pragma unroll
    for (int k = 0; k < (B < 4 ? B : 4); k++) low[k] = (uint32_t)(v >> (k * m)) & lmask;
    if constexpr (B > 4) {
      const uint64_t v2 = join64(w.l2, (p + 4u * m) & 31u);
#pragma unroll
      for (int k = 4; k < B; k++) low[k] = (uint32_t)(v2 >> ((k - 4) * m)) & lmask;
    }
  }
  // the row's digit fields through the LUT, concatenated, then one digit per value
  const uint32_t plan = is_trit ? plan_t : plan_q;
  const uint32_t pd = rel + (is_bits ? 0u : (plan & 0xffu));
  const uint32_t win = __builtin_amdgcn_alignbit(w.dg[1], w.dg[0], pd & 31u);
  const uint32_t fw = is_trit ? 8u : 7u, gb = is_trit ? 10u : 9u, db = is_trit ? 2u : 3u;
  const uint32_t lb = is_trit ? 0u : 256u;
  DigitWord D = 0;
#pragma unroll
  for (int i = 0; i < NF; i++) {
    const uint32_t f = __builtin_amdgcn_ubfe(win, i * fw, (plan >> (16 + 4 * i)) & 15u);
    D |= (DigitWord)lut[lb + f] << (i * gb);
  }
  const DigitWord rowd = D >> ((plan >> 8) & 0xffu);
  const uint32_t dmask = is_bits ? 0u : (is_trit ? 3u : 7u);
  uint32_t u[B];
#pragma unroll
  for (int k = 0; k < B; k++) u[k] = ((((uint32_t)(rowd >> (k * db))) & dmask) << m) | low[k];
#pragma unroll
  for (int i = 0; i < B / 2; i++) d[i] = unzigzag_pk(u[2 * i] | (u[2 * i + 1] << 16), q);
}

template <int B>
__device__ __forceinline__ void decode_row(const uint32_t *gw, uint32_t e, uint32_t plan_t, uint32_t plan_q, int y,
                                           int q, const uint16_t *lut, uint32_t d[B / 2]) {
  RowWords<B> w;
  fetch_row<B>(gw, e, plan_t, plan_q, y, w);
  finish_row<B>(w, e, plan_t, plan_q, y, q, lut, d);
}

// a row of B int16 samples as B/2 packed words
template <int B>
__device__ __forceinline__ void load_row(const int16_t *p, uint32_t x[B / 2]) {
  if constexpr (B == 2) {
    x[0] = *reinterpret_cast<const uint32_t *>(p);
  } else if constexpr (B == 4) {
    const uint2 v = *reinterpret_cast<const uint2 *>(p);
    x[0] = v.x;
    x[1] = v.y;
  } else {
    const uint4 v = *reinterpret_cast<const uint4 *>(p);
    x[0] = v.x;
    x[1] = v.y;
    x[2] = v.z;
    x[3] = v.w;
  }
}

template <int B>
__device__ __forceinline__ void store_row(int16_t *p, const uint32_t x[B / 2]) {
  if constexpr (B == 2) {
    *reinterpret_cast<uint32_t *>(p) = x[0];
  } else if constexpr (B == 4) {
    *reinterpret_cast<uint2 *>(p) = make_uint2(x[0], x[1]);
  } else {
    *reinterpret_cast<uint4 *>(p) = make_uint4(x[0], x[1], x[2], x[3]);
  }
}

// Stores of output that no kernel of the same call reads again, with the
// non-temporal hint when NT: streamed to HBM without displacing what L2 and
// the Infinity Cache hold (the compressed input of the next call).
typedef uint32_t u32x2_t __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
template <bool NT>
__device__ __forceinline__ void put4(int16_t *p, const uint32_t x[4]) {
  if constexpr (NT) {
    const u32x4_t v = {x[0], x[1], x[2], x[3]};
    __builtin_nontemporal_store(v, reinterpret_cast<u32x4_t *>(p));
  } else {
    *reinterpret_cast<uint4 *>(p) = make_uint4(x[0], x[1], x[2], x[3]);
  }
}
template <int B, bool NT>
__device__ __forceinline__ void put_row(int16_t *p, const uint32_t x[B / 2]) {
  if constexpr (!NT) {
    store_row<B>(p, x);
  } else if constexpr (B == 2) {
    __builtin_nontemporal_store(x[0], reinterpret_cast<uint32_t *>(p));
  } else if constexpr (B == 4) {
    const u32x2_t v = {x[0], x[1]};
    __builtin_nontemporal_store(v, reinterpret_cast<u32x2_t *>(p));
  } else {
    put4<true>(p, x);
  }
}

// ---------------------------------------------------------------------------
// whole light field, images layout
// ---------------------------------------------------------------------------

constexpr int kLFThreads = 512;
constexpr int kLFWaves = kLFThreads / 64;
constexpr int kLFHeadWords = 448;     // LDS words before the residual tile (LUT, per-block extents)
constexpr int kStagePad = 8;          // zero words after the staged group words

// LDS words of the whole-field kernel's compact tile: tile_cap slots of
// stored blocks and one zero slot, rounded up to 16 bytes.
__host__ __device__ constexpr int lf_tile_words(int tile_cap, int S) { return ((tile_cap + 1) * (S / 2) + 3) & ~3; }

struct LFArgs {
  const int16_t *rkv;
  const uint32_t *off;
  const uint32_t *srv;
  const uint32_t *sched;      // decode schedule: one record per strip (see build_schedule on the host)
  const uint32_t *strip_off;  // [n_strips+1] word offset of each strip's record
  const uint32_t *order;      // [n_strips] strip of each workgroup, costliest first
  const int32_t *batch;       // [nbatch][kBatchWords] runs of sibling leaves (see internal.h)
  int16_t *out;               // [nv][3][hp][wp]
  int nbx, nv, L, q, wp, hp, nb, nbatch;
  int stage_cap;              // LDS words available for staging the strip
  int vec_store;              // output rows may be stored 16 bytes at a time
  int n_top, key_words;       // key views; LDS words of the strip's key-view rows (0: not staged)
  int tile_cap;               // blocks of the compact residual tile
  int stream_out;             // store the output with the non-temporal hint
};

// A whole block of a known kind (0 plain bits, 1 trit, 2 quint) decoded by one
// lane: d holds the B*B residuals as packed int16 pairs, row-major.  With the
// kind and the row fixed at compile time, every field position except the
// m-dependent low-bit offsets is a constant.
template <int B, int KIND>
__device__ __forceinline__ void decode_block_k(const uint32_t *gw, uint32_t e, int q, const uint16_t *lut,
                                               uint32_t d[B * B / 2]) {
  constexpr int S = B * B;
  constexpr uint32_t HDR = KIND == 0 ? 0u : (KIND == 1 ? Planes<S>::trit : Planes<S>::quint);
  constexpr uint32_t FW = KIND == 1 ? 8u : 7u, GB = KIND == 1 ? 10u : 9u, DB = KIND == 1 ? 2u : 3u;
  constexpr uint32_t LB = KIND == 1 ? 0u : 256u, DMASK = KIND == 1 ? 3u : 7u;
  using DigitWord = std::conditional_t<B == 8, uint64_t, uint32_t>;
  const uint32_t code = e & 31u, rel = e >> 5;
  const uint32_t m = KIND == 0 ? code + 1u : (KIND == 1 ? code - 12u : code - 19u);
  const uint32_t lmask = (1u << m) - 1u;
  if constexpr (B <= 4 && KIND != 0) {
    // Trits and quints at B <= 4: a row's low bits (B*m <= 24) lie in one
    // 32-bit window of two words, and the digit plane (at most 38 bits) is
    // read once, in two or three words, and expanded field by field: every
    // field is looked up once instead of once per row that shares it.
    constexpr uint32_t DPG = KIND == 1 ? 5u : 3u;   // digits per field
    constexpr int NG = (int)((S + DPG - 1) / DPG);
    using AllDigits = std::conditional_t<(KIND == 2 && S > 10), uint64_t, uint32_t>;
    const uint32_t *qd = gw + (rel >> 5);
    const uint32_t sh = rel & 31u;
    uint64_t plane = __builtin_amdgcn_alignbit(qd[1], qd[0], sh);
    if constexpr (HDR > 32) plane |= (uint64_t)__builtin_amdgcn_alignbit(qd[2], qd[1], sh) << 32;
    AllDigits D = 0;
#pragma unroll
    for (int g = 0; g < NG; g++) {
      const uint32_t off = (uint32_t)g * FW;
      const uint32_t wdt = HDR - off < FW ? HDR - off : FW;
      D |= (AllDigits)lut[LB + ((uint32_t)(plane >> off) & ((1u << wdt) - 1u))] << (g * GB);
    }
#pragma unroll
    for (int y = 0; y < B; y++) {
      const uint32_t p = rel + HDR + (uint32_t)(y * B) * m;
      const uint32_t *qr = gw + (p >> 5);
      const uint32_t lo = __builtin_amdgcn_alignbit(qr[1], qr[0], p & 31u);
      uint32_t u[B];
#pragma unroll
      for (int k = 0; k < B; k++)
        u[k] = __builtin_amdgcn_ubfe(lo, (uint32_t)k * m, m) |
               ((((uint32_t)(D >> ((y * B + k) * DB))) & DMASK) << m);
#pragma unroll
      for (int i = 0; i < B / 2; i++) d[y * (B / 2) + i] = unzigzag_pk(u[2 * i] | (u[2 * i + 1] << 16), q);
    }
    return;
  }
#pragma unroll
  for (int y = 0; y < B; y++) {
    uint32_t u[B];
    const uint32_t p = rel + HDR + (uint32_t)(y * B) * m;
    {
      const uint64_t v = window64(gw, p);
#pragma unroll
      for (int k = 0; k < (B < 4 ? B : 4); k++) u[k] = (uint32_t)(v >> (k * m)) & lmask;
      if constexpr (B > 4) {
        const uint64_t v2 = window64(gw, p + 4u * m);
#pragma unroll
        for (int k = 4; k < B; k++) u[k] = (uint32_t)(v2 >> ((k - 4) * m)) & lmask;
      }
    }
    if constexpr (KIND != 0) {
      const uint32_t plan = digit_plan<B>(y, KIND == 1);   // a constant once unrolled
      const uint32_t pd = rel + (plan & 0xffu);
      const uint32_t *qd = gw + (pd >> 5);
      const uint32_t win = __builtin_amdgcn_alignbit(qd[1], qd[0], pd & 31u);
      DigitWord D = 0;
#pragma unroll
      for (int i = 0; i < (B == 8 ? 4 : 2); i++) {
        const uint32_t wdt = (plan >> (16 + 4 * i)) & 15u;
        if (wdt) D |= (DigitWord)lut[LB + ((win >> (i * FW)) & ((1u << wdt) - 1u))] << (i * GB);
      }
      const DigitWord rowd = D >> ((plan >> 8) & 0xffu);
#pragma unroll
      for (int k = 0; k < B; k++) u[k] |= (((uint32_t)(rowd >> (k * DB))) & DMASK) << m;
    }
#pragma unroll
    for (int i = 0; i < B / 2; i++) d[y * (B / 2) + i] = unzigzag_pk(u[2 * i] | (u[2 * i + 1] << 16), q);
  }
}

// A whole block of any kind decoded by one lane, with the generic row
// decoder (one code for the three kinds, the row plans constant).
template <int B>
__device__ __forceinline__ void decode_block(const uint32_t *gw, uint32_t e, int q, const uint16_t *lut,
                                             uint32_t d[B * B / 2]) {
#pragma unroll
  for (int y = 0; y < B; y++)
    decode_row<B>(gw, e, digit_plan<B>(y, true), digit_plan<B>(y, false), y, q, lut, d + y * (B / 2));
}

// n words from global memory into LDS, without a round trip through
// registers: lane i of each wave-wide load writes dst[i0 + i].
__device__ __forceinline__ void lds_copy(uint32_t *dst, const uint32_t *src, uint32_t n, int lane) {
  for (uint32_t i0 = 0; i0 < n; i0 += 64)
    if (i0 + (uint32_t)lane < n)
      __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)(src + i0 + lane),
                                       (__attribute__((address_space(3))) void *)(dst + i0), 4, 0, 0);
}

// A workgroup barrier for data exchanged through LDS only: this wave's LDS
// operations complete before it, but its global stores stay in flight (a
// __syncthreads() would also wait for every outstanding store of the wave,
// and the whole-field kernel's stores need not be visible to other waves).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0); vmcnt and expcnt not waited on
  __builtin_amdgcn_s_barrier();
}

// Tables that every lane of a wave reads at the same address (tree runs,
// chunk records) are read through the scalar unit: a vector load would make
// the wave wait for all of its outstanding stores as well.
typedef const __attribute__((address_space(4))) int32_t *uniform_i32;
__device__ __forceinline__ uniform_i32 as_uniform(const int32_t *p) { return (uniform_i32)p; }

// One chunk of phase B of the whole-field kernel.  sch is the chunk's record
// of the decode schedule (runs, nodes, per-node masks of the stored blocks
// and first tile slots, per-run node positions, directory entries and
// (slot, block) items), in LDS or in global memory; the payload of block j of
// the strip is at pw + s_po[j].  Step (3): every stored block decoded once,
// whole, by one lane, with the decoder of its range kind, into its slot of
// the compact tile; step (4): per sibling run, key-view row + ancestor rows +
// leaf row (absent blocks add nothing), stored 16 bytes per lane.
template <int B, bool KEYS, bool TAB>
__device__ __forceinline__ void lf_chunk(const LFArgs &a, const uint32_t *sch, const uint32_t *pw,
                                         const uint32_t *s_po, uint32_t *tile, const uint32_t *keys,
                                         uint32_t *s_tab, const uint16_t *lut, int tid, int wave, int lane, int so,
                                         int jq, int bx0, int nact, bool wide, uint64_t lane_off, uint32_t vstride,
                                         int by, int c) {
  constexpr int S = B * B, NBLK = 64 / B, H = B / 2, PB = 8 / B;
  // the chunk's header fields, the same for every lane (made scalar)
  const int q0 = __builtin_amdgcn_readfirstlane((int)sch[0]), nq = __builtin_amdgcn_readfirstlane((int)sch[1]);
  const int nn = __builtin_amdgcn_readfirstlane((int)sch[2]);
  const uint32_t n0 = __builtin_amdgcn_readfirstlane(sch[3]), n01 = __builtin_amdgcn_readfirstlane(sch[4]);
  const uint32_t n = __builtin_amdgcn_readfirstlane(sch[5]);
  const uint32_t *ents = sch + 6 + nn + (nn + 1) / 2 + 3 * nq;
  const uint16_t *items = reinterpret_cast<const uint16_t *>(ents + n);
  // the gather's table (per-node masks and first slots, per-run node
  // positions): read where the schedule is (LDS in the staging tiers), or,
  // with TAB, copied from global memory into LDS during the decode, so that
  // the gather issues no vector load (each would wait for the wave's
  // outstanding stores)
  const uint32_t *tab = sch + 6;
  if constexpr (TAB) {
    const int tw = nn + (nn + 1) / 2 + 3 * nq;
    for (int w0 = wave * 64; w0 < tw; w0 += kLFThreads)
      if (w0 + lane < tw)
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)(sch + 6 + w0 + lane),
                                         (__attribute__((address_space(3))) void *)(s_tab + w0), 4, 0, 0);
    tab = s_tab;
  }
  const uint32_t *masks = tab;
  const uint16_t *firsts = reinterpret_cast<const uint16_t *>(masks + nn);
  const uint32_t *runs = masks + nn + (nn + 1) / 2;
  // (3) decode; the three kinds are laid end to end, so a wave mostly sees one kind.
  // A lane's next entry is requested before its current block's payload, so
  // the two reads overlap.
  uint32_t e_nx = 0, t_nx = 0;
  if ((uint32_t)tid < n) {
    e_nx = ents[tid];
    t_nx = items[tid];
  }
  for (uint32_t it = tid; it < n; it += kLFThreads) {
    const uint32_t e = e_nx, t = t_nx;
    if (it + kLFThreads < n) {
      e_nx = ents[it + kLFThreads];
      t_nx = items[it + kLFThreads];
    }
    const uint32_t *gw = pw + s_po[t & 31u];
    uint32_t d[S / 2];
    if (it < n0) decode_block_k<B, 0>(gw, e, a.q, lut, d);
    else if (it < n01) decode_block_k<B, 1>(gw, e, a.q, lut, d);
    else decode_block_k<B, 2>(gw, e, a.q, lut, d);
    uint32_t *dst = tile + (t >> 5) * (S / 2);
    if constexpr (S / 2 >= 4) {
#pragma unroll
      for (int w = 0; w < S / 2; w += 4)
        *reinterpret_cast<uint4 *>(dst + w) = make_uint4(d[w], d[w + 1], d[w + 2], d[w + 3]);
    } else {
      *reinterpret_cast<uint2 *>(dst) = make_uint2(d[0], d[1]);
    }
  }
  if constexpr (TAB) __builtin_amdgcn_s_waitcnt(0x0f70);   // vmcnt(0): the table copies have landed
  lds_barrier();
  // (4) gather and store.  A wave takes two runs at a time, one per half; a
  // lane owns one sibling of its run and one 16-byte segment (PB blocks) of
  // the strip's rows, and walks the B rows of its blocks: each node's tile
  // slots are found once per lane, and an absent block reads the zeroed slot
  // at the end of the tile (no masking).  Gather issue goes first; the
  // decode of a workgroup sharing the compute unit fills the gaps.
  __builtin_amdgcn_s_setprio(2);
  const int L = a.L;
  const int half = lane >> 5;
  const uint32_t zslot = (uint32_t)a.tile_cap;       // the zeroed slot
  const int pairs = (nq + 1) / 2, per = (pairs + kLFWaves - 1) / kLFWaves;
  // tile words of this lane's block k of a node (mask mk of its stored
  // blocks, first slot f)
  auto slot_of = [&](uint32_t mk, uint32_t f, int k) -> const uint32_t * {
    const uint32_t j = (uint32_t)(jq * PB + k);
    const uint32_t s = ((mk >> j) & 1u) ? f + (uint32_t)__popc(mk & ((1u << j) - 1u)) : zslot;
    return tile + s * (S / 2);
  };
  for (int qp = wave * per; qp < min(pairs, wave * per + per); qp++) {
    const int q_a = 2 * qp, q_b = min(2 * qp + 1, nq - 1);
    const uniform_i32 ra = as_uniform(a.batch + (size_t)(q0 + q_a) * lfc::kBatchWords);
    const uniform_i32 rb = as_uniform(a.batch + (size_t)(q0 + q_b) * lfc::kBatchWords);
    // both records through the scalar unit (each field made wave-uniform
    // before the per-half choice, so that the choice is not moved into the
    // address of a vector load)
    int fa[6], fb[6];
#pragma unroll
    for (int k = 0; k < 6; k++) {
      fa[k] = __builtin_amdgcn_readfirstlane(ra[k]);
      fb[k] = __builtin_amdgcn_readfirstlane(rb[k]);
    }
    const int qi = half ? q_b : q_a;
    const bool run_live = !half || 2 * qp + 1 < nq;
    const int nsib = half ? fb[0] : fa[0], root = half ? fb[5] : fa[5];
    const int va = so == 0 ? fa[1] : (so == 1 ? fa[2] : (so == 2 ? fa[3] : fa[4]));
    const int vb = so == 0 ? fb[1] : (so == 1 ? fb[2] : (so == 2 ? fb[3] : fb[4]));
    const int vi = half ? vb : va;
    const bool live = run_live && so < nsib;
    // key-view rows
    uint32_t x[B][4];
    if constexpr (KEYS) {
#pragma unroll
      for (int y = 0; y < B; y++) {
        const uint4 k4 = reinterpret_cast<const uint4 *>(keys)[(((root * B + y) * NBLK + jq * PB) * H) / 4];
        x[y][0] = k4.x;
        x[y][1] = k4.y;
        x[y][2] = k4.z;
        x[y][3] = k4.w;
      }
    } else {
#pragma unroll
      for (int y = 0; y < B; y++) {
#pragma unroll
        for (int w = 0; w < 4; w++) x[y][w] = 0;
#pragma unroll
        for (int k = 0; k < PB; k++)
          if (k < nact)
            load_row<B>(a.rkv + ((size_t)(root * a.nb + by * a.nbx + bx0 + k) * 3 + c) * S + y * B, x[y] + k * H);
      }
    }
    // node rows added to every row of the lane's blocks
    auto add_node = [&](int ln) {
      const uint32_t mk = masks[ln], f = firsts[ln];
#pragma unroll
      for (int k = 0; k < PB; k++) {
        const uint32_t *t = slot_of(mk, f, k);
#pragma unroll
        for (int y = 0; y < B; y++) {
          if constexpr (H == 1) {
            x[y][k] = add_pk(x[y][k], t[y]);
          } else if constexpr (H == 2) {
            const uint2 v = *reinterpret_cast<const uint2 *>(t + y * 2);
            x[y][2 * k] = add_pk(x[y][2 * k], v.x);
            x[y][2 * k + 1] = add_pk(x[y][2 * k + 1], v.y);
          } else {
            const uint4 v = *reinterpret_cast<const uint4 *>(t + y * 4);
            x[y][0] = add_pk(x[y][0], v.x);
            x[y][1] = add_pk(x[y][1], v.y);
            x[y][2] = add_pk(x[y][2], v.z);
            x[y][3] = add_pk(x[y][3], v.w);
          }
        }
      }
    };
    const uint32_t w0 = runs[3 * qi], w1 = runs[3 * qi + 1], w2 = runs[3 * qi + 2];
    const int anc_ln[4] = {(int)(w0 >> 16), (int)(w1 & 0xFFFFu), (int)(w1 >> 16), (int)(w2 & 0xFFFFu)};
#pragma unroll
    for (int k = 0; k < 4; k++)
      if (k < L - 2) add_node(anc_ln[k]);
    add_node((int)(w0 & 0xFFFFu) + (live ? so : 0));
    if (!live) continue;
    int16_t *dst = a.out + ((uint64_t)(uint32_t)vi * vstride + lane_off);
    // separate loops, so that the 16-byte stores stay whole
    if (wide && a.stream_out) {
#pragma unroll
      for (int y = 0; y < B; y++) put4<true>(dst + (size_t)y * a.wp, x[y]);
    } else if (wide) {
#pragma unroll
      for (int y = 0; y < B; y++) put4<false>(dst + (size_t)y * a.wp, x[y]);
    } else if (nact > 0) {
#pragma unroll
      for (int y = 0; y < B; y++)
#pragma unroll
        for (int k = 0; k < PB; k++)
          if (k < nact) {
            if (a.stream_out) put_row<B, true>(dst + (size_t)y * a.wp + k * B, x[y] + k * H);
            else put_row<B, false>(dst + (size_t)y * a.wp + k * B, x[y] + k * H);
          }
    }
  }
  __builtin_amdgcn_s_setprio(0);
  lds_barrier();
}

// One workgroup = one channel c, one row of blocks by, one strip of 64/B
// consecutive blocks (64 pixels).  Phase A copies into LDS what fits of the
// strip's data: its groups and its decode schedule (tier 1), else the
// schedule only (tier 2: payload read through bit windows from global
// memory), else nothing (tier 3), plus the strip's key-view rows.  Phase B
// walks the strip's chunks (runs of sibling leaves in serial order whose
// stored blocks fit the compact tile): decode every stored residual block of
// the chunk once into the tile, then write the chunk's leaves (key view +
// ancestors + leaf), 16 bytes per lane.
// (B <= 4: at most 80 VGPRs, six waves per SIMD, so three workgroups share a
// compute unit whenever their LDS fits; B = 8 keeps its registers)
template <int B>
__global__ __launch_bounds__(kLFThreads, B <= 4 ? 6 : 1) void k_decode_lf(LFArgs a) {
  constexpr int S = B * B, NBLK = 64 / B, H = B / 2;
  constexpr int PB = 8 / B;                            // blocks per 16-byte row segment (1 for B = 8)
  extern __shared__ uint32_t smem[];
  uint16_t *lut = reinterpret_cast<uint16_t *>(smem);  // 384 x u16 = 192 words
  uint32_t *s_o0 = smem + 192;                         // group start word in the SRV section
  uint32_t *s_len = smem + 256;                        // group length in words
  uint32_t *s_wo = smem + 320;                         // staged group words
  uint32_t *s_cnt = smem + 384;                        // [0] tier, [1] staged group words, [2] schedule words
  uint32_t *tile = smem + kLFHeadWords;                // compact tile: [tile_cap + 1][S/2], the last slot zero
  uint32_t *keys = tile + lf_tile_words(a.tile_cap, S); // [n_top][B][NBLK][H]
  uint32_t *s_tab = keys + a.key_words;                 // a chunk's gather table (strips read from global memory)
  uint32_t *stage = s_tab + lfc::kLFTabWords;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  // the workgroup's strip (strips are taken costliest first, so the last
  // workgroups to start are short ones)
  // (its order entry: the strip, its schedule, its groups; one load)
  constexpr int OW = lfc::order_words(B);
  const uint32_t *ent = a.order + (size_t)((blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x) * OW;
  const uniform_i32 uent = as_uniform(reinterpret_cast<const int32_t *>(ent));
  const int st = uent[0];
  const int sx = st % (int)gridDim.x, by = (st / (int)gridDim.x) % (int)gridDim.y, c = st / ((int)gridDim.x * (int)gridDim.y);
  const uint32_t sched0 = (uint32_t)uent[1], sched_len = (uint32_t)uent[2];
  // the LUT from its table (a copy straight into LDS)
  if (tid < kLutEntries / 2) __builtin_amdgcn_global_load_lds(
      (const __attribute__((address_space(1))) void *)(kLutTable.w + tid),
      (__attribute__((address_space(3))) void *)(smem + (tid & ~63)), 4, 0, 0);
  if (tid < S / 2) tile[a.tile_cap * (S / 2) + tid] = 0u;   // the slot of every absent block
  if (tid < 64) {
    // wave 0: the strip's group offsets and lengths, their exclusive prefix
    // sum (a wave scan) and the staging tier
    uint32_t o0 = 0, len = 0;
    if (lane < NBLK) {
      o0 = ent[4 + lane];
      len = ent[4 + NBLK + lane];
    }
    uint32_t incl = len;
#pragma unroll
    for (int d = 1; d < NBLK; d <<= 1) {
      const uint32_t v = __shfl_up(incl, d);
      if (lane >= d) incl += v;
    }
    const uint32_t words = __shfl(incl, NBLK - 1);
    if (lane < NBLK) {
      s_o0[lane] = o0;
      s_len[lane] = len;
      s_wo[lane] = incl - len;
    }
    if (lane == 0) {
      // tier 1: [group words][pad][schedule]; tier 2: [schedule]
      const uint32_t tier = words + kStagePad + sched_len <= (uint32_t)a.stage_cap ? 1u
                            : (sched_len <= (uint32_t)a.stage_cap ? 2u : 3u);
      s_cnt[0] = tier;
      s_cnt[1] = tier == 1u ? words : 0u;
      s_cnt[2] = tier == 1u ? words + kStagePad : 0u;
    }
  }
  __syncthreads();
  const uint32_t tier = s_cnt[0], sched_at = s_cnt[2];
  // every copy goes straight from global memory to LDS, all in flight at once
  if (tier == 1u)
    for (int j = wave; j < NBLK; j += kLFWaves)
      if (s_len[j]) lds_copy(stage + s_wo[j], a.srv + s_o0[j], s_len[j], lane);
  if (tier < 3u) {
    // the schedule, split over the waves in pieces of whole 64-word rows
    const uint32_t rows = (sched_len + 63) / 64, per = (rows + kLFWaves - 1) / kLFWaves;
    const uint32_t r0 = min(rows, (uint32_t)wave * per), r1 = min(rows, r0 + per);
    if (r1 > r0) lds_copy(stage + sched_at + r0 * 64, a.sched + sched0 + r0 * 64, min(sched_len, r1 * 64) - r0 * 64, lane);
  }
  if (a.key_words) {
    // the strip's key-view rows, laid out as the tile: [root][row][block][H]
    const uint32_t *rk = reinterpret_cast<const uint32_t *>(a.rkv);
    for (int t0 = wave * 64; t0 < a.key_words; t0 += kLFThreads) {
      const int t = t0 + lane, h = t % H, j = (t / H) % NBLK, y = (t / (H * NBLK)) % B, r = t / (H * NBLK * B);
      const int bx = sx * NBLK + j;
      if (t < a.key_words && bx < a.nbx)
        __builtin_amdgcn_global_load_lds(
            (const __attribute__((address_space(1))) void *)(rk + ((size_t)(r * a.nb + by * a.nbx + bx) * 3 + c) *
                                                                  (S / 2) + y * H + h),
            (__attribute__((address_space(3))) void *)(keys + t0), 4, 0, 0);
    }
  }
  __builtin_amdgcn_s_waitcnt(0);
  if (tier == 1u && tid < kStagePad) stage[s_cnt[1] + tid] = 0;
  __syncthreads();

  const uint32_t vstride = 3u * (uint32_t)a.hp * (uint32_t)a.wp;
  const uint64_t cplane = (uint64_t)c * a.hp * a.wp;
  if (a.L == 1) {
    // no residual levels: every view is a stored key view
    const int j = lane % NBLK, y = lane / NBLK, bx = sx * NBLK + j;
    if (bx >= a.nbx) return;
    const int b = by * a.nbx + bx;
    const int per = (a.nbatch + kLFWaves - 1) / kLFWaves;
    for (int qb = wave * per; qb < min(a.nbatch, wave * per + per); qb++) {
      const uniform_i32 rec = as_uniform(a.batch + (size_t)qb * lfc::kBatchWords);
      uint32_t x[H];
      load_row<B>(a.rkv + ((size_t)(rec[5] * a.nb + b) * 3 + c) * S + y * B, x);
      int16_t *dst = a.out + (size_t)rec[1] * vstride + cplane + (size_t)(by * B + y) * a.wp + bx * B;
      if (a.stream_out) put_row<B, true>(dst, x);
      else put_row<B, false>(dst, x);
    }
    return;
  }
  // store-side lane mapping: run of the wave's pair (lane / 32), sibling in
  // the run, segment of PB blocks (16 bytes of each of the B rows)
  const int so = (lane >> 3) & 3, jq = lane & 7;
  const int bx0 = sx * NBLK + jq * PB;
  const int nact = max(0, min(PB, a.nbx - bx0));       // blocks of the segment inside the image
  const bool wide = nact == PB && a.vec_store;          // a 16-byte store is aligned
  const uint64_t lane_off = cplane + (uint64_t)(by * B) * a.wp + (uint64_t)bx0 * B;
  const uint32_t *gsched = a.sched + sched0;
  const uint32_t *lsched = stage + sched_at;
  const int nck = (int)(tier < 3u ? lsched[0] : gsched[0]);
  // one code path per staging tier and key-row placement, so that no path
  // carries loads it never issues
  auto chunks = [&](auto keys_staged) {
    constexpr bool K = decltype(keys_staged)::value;
    for (int ci = 0; ci < nck; ci++) {
      if (tier == 1u)
        lf_chunk<B, K, false>(a, lsched + lsched[1 + ci], stage, s_wo, tile, keys, s_tab, lut, tid, wave, lane, so, jq,
                              bx0, nact, wide, lane_off, vstride, by, c);
      else if (tier == 2u)
        lf_chunk<B, K, false>(a, lsched + lsched[1 + ci], a.srv, s_o0, tile, keys, s_tab, lut, tid, wave, lane, so, jq,
                              bx0, nact, wide, lane_off, vstride, by, c);
      else
        lf_chunk<B, K, true>(a, gsched + gsched[1 + ci], a.srv, s_o0, tile, keys, s_tab, lut, tid, wave, lane, so, jq,
                             bx0, nact, wide, lane_off, vstride, by, c);
    }
  };
  if (a.key_words) chunks(std::true_type{});
  else chunks(std::false_type{});
}

// ---------------------------------------------------------------------------
// random access: one (view, block) at a time through the directory
// ---------------------------------------------------------------------------

struct RAArgs {
  const int16_t *rkv;
  const uint32_t *off;
  const uint32_t *srv;
  const uint32_t *dbase;
  const uint32_t *poff;
  const int32_t *path;
  const int32_t *root;
  int nb, nbx, nv, nbw, L, q;
  const uint32_t *dir2;   // [nb][nbw][3] (bitmap word, dbase entry) pairs
};

// Row y of block b, channel c, of view vi (Alg. 2): key-view row plus the
// residual rows of the view's ancestors on levels L-2 down to stop (0: the
// view itself; a higher stop is progressive decompression, Sec. 3.6), as B/2
// packed int16 pairs.
template <int B>
__device__ __forceinline__ void gather_row(const RAArgs &a, int vi, int b, int c, int y, int stop, uint32_t plan_t,
                                           uint32_t plan_q, const uint16_t *lut, uint32_t x[B / 2]) {
  constexpr int S = B * B;
  const int root = a.root[vi];
  load_row<B>(a.rkv + ((size_t)(root * a.nb + b) * 3 + c) * S + y * B, x);
  const int g = 3 * b + c;
  const uint32_t o0 = a.off[g], o1 = a.off[g + 1];
  if (o0 == o1) return;
  const uint32_t *gw = a.srv + o0;
  const int depth = a.L - 1;
  for (int l = depth - 1; l >= stop; --l) {
    const int s = a.path[vi * depth + l];
    // the bitmap word and the directory index of its first stored node, read together
    const uint2 bd = *reinterpret_cast<const uint2 *>(a.dir2 + (((size_t)b * a.nbw + (s >> 5)) * 3 + c) * 2);
    const uint32_t bm = bd.x;
    const uint32_t bit = (uint32_t)s & 31u;
    if ((bm >> bit) & 1u) {
      const uint32_t idx = bd.y + __popc(bm & ((1u << bit) - 1u));
      uint32_t d[B / 2];
      decode_row<B>(gw, a.poff[idx], plan_t, plan_q, y, a.q, lut, d);
#pragma unroll
      for (int i = 0; i < B / 2; i++) x[i] = add_pk(x[i], d[i]);
    }
  }
}

struct BlocksArgs {
  RAArgs ra;
  const int32_t *req;  // [n][2] or null
  int16_t *out;        // [n][3][S]
  int32_t *err;
  int64_t n;
  int stop;            // lowest tree level whose residuals are added
};

template <int B>
__global__ __launch_bounds__(kThreads) void k_decode_blocks(BlocksArgs a) {
  constexpr int S = B * B, LPR = 3 * B, RPW = 64 / LPR;
  __shared__ uint16_t lut[kLutEntries];
  for (int t = threadIdx.x; t < kLutEntries; t += kThreads) lut[t] = lut_entry(t);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * kThreads + threadIdx.x) >> 6;
  const int slot = lane / LPR, sub = lane % LPR;
  if (slot >= RPW) return;
  const int64_t r = wave * RPW + slot;
  if (r >= a.n) return;
  const int c = sub / B, y = sub % B;
  int vi, b;
  if (a.req) {
    vi = a.req[2 * r];
    b = a.req[2 * r + 1];
  } else {
    vi = (int)(r / a.ra.nb);
    b = (int)(r % a.ra.nb);
  }
  uint32_t x[B / 2];
  if (vi < 0 || vi >= a.ra.nv || b < 0 || b >= a.ra.nb) {
    if (sub == 0) atomicOr(a.err, 1);
#pragma unroll
    for (int i = 0; i < B / 2; i++) x[i] = 0;
  } else {
    gather_row<B>(a.ra, vi, b, c, y, a.stop, digit_plan<B>(y, true), digit_plan<B>(y, false), lut, x);
  }
  store_row<B>(a.out + ((size_t)r * 3 + c) * S + y * B, x);
}

// Random access over many light fields of one block size in one launch:
// request r = (light field, view, block) indexes a table of the light
// fields' device tables; otherwise as k_decode_blocks.
struct MultiArgs {
  const RAArgs *lfs;
  int32_t n_lf;
  const int32_t *req;  // [n][3]
  int16_t *out;        // [n][3][S]
  int32_t *err;
  int64_t n;
};

template <int B>
__global__ __launch_bounds__(kThreads) void k_decode_multi(MultiArgs a) {
  constexpr int S = B * B, LPR = 3 * B, RPW = 64 / LPR;
  __shared__ uint16_t lut[kLutEntries];
  for (int t = threadIdx.x; t < kLutEntries; t += kThreads) lut[t] = lut_entry(t);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * kThreads + threadIdx.x) >> 6;
  const int slot = lane / LPR, sub = lane % LPR;
  if (slot >= RPW) return;
  const int64_t r = wave * RPW + slot;
  if (r >= a.n) return;
  const int c = sub / B, y = sub % B;
  const int li = a.req[3 * r], vi = a.req[3 * r + 1], b = a.req[3 * r + 2];
  uint32_t x[B / 2];
  if (li < 0 || li >= a.n_lf || vi < 0 || vi >= a.lfs[li].nv || b < 0 || b >= a.lfs[li].nb) {
    if (sub == 0) atomicOr(a.err, 1);
#pragma unroll
    for (int i = 0; i < B / 2; i++) x[i] = 0;
  } else {
    const RAArgs la = a.lfs[li];   // the light field's record, read once
    gather_row<B>(la, vi, b, c, y, 0, digit_plan<B>(y, true), digit_plan<B>(y, false), lut, x);
  }
  store_row<B>(a.out + ((size_t)r * 3 + c) * S + y * B, x);
}

// ---------------------------------------------------------------------------
// novel views: footprint decode into LDS, then quadrilinear interpolation
// ---------------------------------------------------------------------------

struct RenderArgs {
  RAArgs ra;
  const lfc_view *views;
  float *out;  // [n][3][ho][wo]
  int wo, ho, U, V, W, H, TX, TY, fbx_max, fby_max;
  float disp;  // focal disparity: image-plane shift per unit of camera-grid offset
};

// lower grid index, upper index and fraction of x on [0, n-1], after clamping
__device__ __forceinline__ void cell(float x, int n, int &i0, int &i1, float &f) {
  x = fminf(fmaxf(x, 0.0f), (float)(n - 1));
  if (n == 1) {
    i0 = i1 = 0;
    f = 0.0f;
    return;
  }
  int i = (int)floorf(x);
  i = min(max(i, 0), n - 2);
  i0 = i;
  i1 = i + 1;
  f = x - (float)i;
}

__device__ __forceinline__ float lerpf(float a, float b, float f) { return a + f * (b - a); }

__device__ __forceinline__ int32_t lo16(uint32_t w) { return (int32_t)(int16_t)(w & 0xFFFFu); }
__device__ __forceinline__ int32_t hi16(uint32_t w) { return (int32_t)(int16_t)(w >> 16); }

// The residual-block entry (payload offset << 5 | code) of node s in group g,
// or kAbsent, through the directory built at initialisation.
__device__ __forceinline__ uint32_t locate(const RAArgs &a, int g, int s, const uint32_t **gw_out) {
  const uint32_t o0 = a.off[g], o1 = a.off[g + 1];
  if (o0 == o1) return kAbsent;
  const uint2 bd = *reinterpret_cast<const uint2 *>(a.dir2 + ((size_t)(g / 3 * a.nbw + (s >> 5)) * 3 + g % 3) * 2);
  const uint32_t bm = bd.x, bit = (uint32_t)s & 31u;
  if (!((bm >> bit) & 1u)) return kAbsent;
  *gw_out = a.srv + o0;
  return a.poff[bd.y + __popc(bm & ((1u << bit) - 1u))];
}

// Threads of a render-tile workgroup: 8 waves, so that a tile's footprint
// decode (a chain of dependent reads per level) and its interpolation run
// in half the passes of a 4-wave workgroup at the same LDS per tile.
constexpr int kRenderThreads = 512;

// One workgroup per (view, output tile).  The tile's source footprint in the
// four nearest views is reconstructed in LDS: first the key-view rows, then,
// level by level, every distinct stored residual block of the footprint is
// located, decoded whole by one lane and added for each of the four views
// whose path passes through that node (neighbouring views often share
// ancestors).  The sums are converted to RGB (inverse YCoCg-R, clamped) in
// place, then every output pixel interpolates its 16 taps in FP32.
// Inverse YCoCg-R (Sec. 4) of one sample, clamped to 8 bits, packed R | G << 8 | B << 16.
__device__ __forceinline__ uint32_t rgb_pack(int32_t yv, int32_t co, int32_t cg) {
  const int32_t t = yv - (cg >> 1);
  const int32_t G = cg + t;
  const int32_t Bc = t - (co >> 1);
  const int32_t R = Bc + co;
  return (uint32_t)min(max(R, 0), 255) | ((uint32_t)min(max(G, 0), 255) << 8) | ((uint32_t)min(max(Bc, 0), 255) << 16);
}

// The quadrilinear interpolation of one output pixel from its 16 taps
// P[k][0..3] = (y0,x0), (y0,x1), (y1,x0), (y1,x1) of view k = 0: (u0, v0),
// 1: (u1, v0), 2: (u0, v1), 3: (u1, v1); lerps in s, t, v, u order.
// Camera-plane position (clamped to the grid) and the image-plane shift of
// source view k (0: lower column/row, 1: upper) for focal disparity d: a
// novel camera focused at disparity d samples source camera (iu, jv) at
// (s + d (iu - u), t + d (jv - v)).
// FOCAL false compiles the plain render, where every source view shares one
// footprint and one set of fractions.
template <bool FOCAL>
__device__ __forceinline__ float focal_shift(float d, float x, int n, int i) {
#pragma clang fp contract(off)
  if constexpr (!FOCAL) return 0.0f;
  return d * ((float)i - fminf(fmaxf(x, 0.0f), (float)(n - 1)));
}

// Source-image position of output pixel X: each operation rounded on its
// own (no fused multiply-add), so every renderer samples the same positions.
__device__ __forceinline__ float src_pos(float s, int X, float scale) {
#pragma clang fp contract(off)
  return s + ((float)X + 0.5f) * scale - 0.5f;
}

// x / 255 for 0 <= x <= 255, rounded as the IEEE quotient: the product with
// the rounded reciprocal, corrected by one fused residual step (equal to the
// division for every float of the range, checked on the host by
// tests/arith_identities.c; negative inputs mirror it); three VALU operations
// instead of a full division.
__device__ __forceinline__ float div255(float x) {
  constexpr float r = 1.0f / 255.0f;
  const float q = x * r;
  return __builtin_fmaf(__builtin_fmaf(-q, 255.0f, x), r, q);
}

// quadrilinear interpolation of the 16 RGB taps P[view][tap] (taps 00, 01,
// 10, 11 of each view, at that view's fractions fs[k], ft[k])
__device__ __forceinline__ void interp_store(const uint32_t P[4][4], const float fs[4], const float ft[4], float fu,
                                             float fv, float *o, size_t plane) {
#pragma unroll
  for (int ch = 0; ch < 3; ch++) {
    float lt[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const float p00 = (float)((P[k][0] >> (8 * ch)) & 255u), p01 = (float)((P[k][1] >> (8 * ch)) & 255u);
      const float p10 = (float)((P[k][2] >> (8 * ch)) & 255u), p11 = (float)((P[k][3] >> (8 * ch)) & 255u);
      lt[k] = lerpf(lerpf(p00, p01, fs[k]), lerpf(p10, p11, fs[k]), ft[k]);
    }
    const float lv0 = lerpf(lt[0], lt[2], fv), lv1 = lerpf(lt[1], lt[3], fv);
    o[ch * plane] = div255(lerpf(lv0, lv1, fu));
  }
}

// One output tile (tile column tbx, tile row tby) of view vw into outn
// ([3][ho][wo] floats); smem holds the LUT and the footprint accumulators.
template <int B, bool FOCAL>
__device__ __forceinline__ void render_tile(const RenderArgs &a, const lfc_view vw, float *outn, int tbx, int tby,
                                            uint32_t *smem) {
  constexpr int S = B * B, SLOT = 3 * S / 2;   // words per (view, block): 3 channels of packed int16
  uint16_t *lut = reinterpret_cast<uint16_t *>(smem);
  uint32_t *acc = smem + kLutEntries / 2;       // [4][fbx_max*fby_max][SLOT]
  const int tid = threadIdx.x;
  for (int t = tid; t < kLutEntries; t += kRenderThreads) lut[t] = lut_entry(t);
  int iu0, iu1, jv0, jv1;
  float fu, fv;
  cell(vw.u, a.U, iu0, iu1, fu);
  cell(vw.v, a.V, jv0, jv1, fv);
  const float sxs = (float)a.W / (float)a.wo, tys = (float)a.H / (float)a.ho;
  const int tx0 = tbx * a.TX, ty0 = tby * a.TY;
  const int tx1 = min(tx0 + a.TX, a.wo) - 1, ty1 = min(ty0 + a.TY, a.ho) - 1;
  int vis[4];
  vis[0] = jv0 * a.U + iu0;
  vis[1] = jv0 * a.U + iu1;
  vis[2] = jv1 * a.U + iu0;
  vis[3] = jv1 * a.U + iu1;
  // per source view: image-plane shift (focal disparity) and the tile's
  // source footprint, one pixel wider on each side than needed
  float shx[4], shy[4];
  int fbx0[4], fby0[4], FBX[4], FBY[4], FB[4];
  int FBmax = 0;
#pragma unroll
  for (int k = 0; k < 4; k++) {
    shx[k] = focal_shift<FOCAL>(a.disp, vw.u, a.U, (k & 1) ? iu1 : iu0);
    shy[k] = focal_shift<FOCAL>(a.disp, vw.v, a.V, (k & 2) ? jv1 : jv0);
    const float sa = fminf(fmaxf(src_pos(vw.s, tx0, sxs) + shx[k], 0.0f), (float)(a.W - 1));
    const float sb = fminf(fmaxf(src_pos(vw.s, tx1, sxs) + shx[k], 0.0f), (float)(a.W - 1));
    const float ta = fminf(fmaxf(src_pos(vw.t, ty0, tys) + shy[k], 0.0f), (float)(a.H - 1));
    const float tb = fminf(fmaxf(src_pos(vw.t, ty1, tys) + shy[k], 0.0f), (float)(a.H - 1));
    const int xlo = max((int)floorf(sa) - 1, 0), xhi = min((int)floorf(sb) + 2, a.W - 1);
    const int ylo = max((int)floorf(ta) - 1, 0), yhi = min((int)floorf(tb) + 2, a.H - 1);
    fbx0[k] = xlo / B;
    fby0[k] = ylo / B;
    FBX[k] = min(xhi / B - fbx0[k] + 1, a.fbx_max);
    FBY[k] = min(yhi / B - fby0[k] + 1, a.fby_max);
    FB[k] = FBX[k] * FBY[k];
    FBmax = max(FBmax, FB[k]);
  }
  const int FBM = a.fbx_max * a.fby_max;
  const int depth = a.ra.L - 1;
  __syncthreads();

  // (1) key-view rows: item = (view k, block, channel, row)
  for (int it = tid; it < 4 * FBmax * 3 * B; it += kRenderThreads) {
    const int y = it % B, r1 = it / B, c = r1 % 3, r2 = r1 / 3, bb = r2 % FBmax, k = r2 / FBmax;
    if (bb >= FB[k]) continue;
    const int b = (fby0[k] + bb / FBX[k]) * a.ra.nbx + fbx0[k] + bb % FBX[k];
    uint32_t x[B / 2];
    load_row<B>(a.ra.rkv + ((size_t)(a.ra.root[vis[k]] * a.ra.nb + b) * 3 + c) * S + y * B, x);
#pragma unroll
    for (int h = 0; h < B / 2; h++) acc[(k * FBM + bb) * SLOT + c * (S / 2) + y * (B / 2) + h] = x[h];
  }
  __syncthreads();

  // (2) residual levels, one at a time (each (view, block, channel) slot gets
  // one block per level, so the adds never race)
  for (int l = depth - 1; l >= 0; --l) {
    int node[4], owner[4];
#pragma unroll
    for (int k = 0; k < 4; k++) node[k] = a.ra.path[vis[k] * depth + l];
#pragma unroll
    for (int k = 0; k < 4; k++) {
      // views with one ancestor share its decoded blocks when their
      // footprints coincide (no focal shift)
      owner[k] = k;
      if (!FOCAL)
        for (int k2 = k - 1; k2 >= 0; --k2)
          if (node[k2] == node[k]) owner[k] = k2;
    }
    for (int it = tid; it < 4 * FBmax * 3; it += kRenderThreads) {
      const int c = it % 3, r1 = it / 3, bb = r1 % FBmax, k = r1 / FBmax;
      if (owner[k] != k || bb >= FB[k]) continue;
      const int b = (fby0[k] + bb / FBX[k]) * a.ra.nbx + fbx0[k] + bb % FBX[k];
      const uint32_t *gw = nullptr;
      const uint32_t e = locate(a.ra, 3 * b + c, node[k], &gw);
      if (e == kAbsent) continue;
      uint32_t d[S / 2];
      decode_block<B>(gw, e, a.ra.q, lut, d);
#pragma unroll
      for (int k2 = 0; k2 < 4; k2++) {
        if (owner[k2] != k) continue;
        uint32_t *slot = acc + (k2 * FBM + bb) * SLOT + c * (S / 2);
#pragma unroll
        for (int h = 0; h < S / 2; h++) slot[h] = add_pk(slot[h], d[h]);
      }
    }
    __syncthreads();
  }

  // (3) YCoCg-R -> RGB in place: item = (view, block)
  for (int it = tid; it < 4 * FBmax; it += kRenderThreads) {
    const int k = it / FBmax, bb = it % FBmax;
    if (bb >= FB[k]) continue;
    uint32_t *slot = acc + (k * FBM + bb) * SLOT;
    uint32_t v[SLOT];
#pragma unroll
    for (int w = 0; w < SLOT; w++) v[w] = slot[w];
#pragma unroll
    for (int i = 0; i < S; i++) {
      const int32_t yv = (i & 1) ? hi16(v[i / 2]) : lo16(v[i / 2]);
      const int32_t co = (i & 1) ? hi16(v[S / 2 + i / 2]) : lo16(v[S / 2 + i / 2]);
      const int32_t cg = (i & 1) ? hi16(v[S + i / 2]) : lo16(v[S + i / 2]);
      slot[i] = rgb_pack(yv, co, cg);
    }
  }
  __syncthreads();

  // (4) quadrilinear interpolation of every output pixel of the tile
  const size_t plane = (size_t)a.ho * a.wo;
  for (int p = tid; p < a.TX * a.TY; p += kRenderThreads) {
    const int X = tx0 + p % a.TX, Yp = ty0 + p / a.TX;
    if (X >= a.wo || Yp >= a.ho) continue;
    const float sx = src_pos(vw.s, X, sxs), ty = src_pos(vw.t, Yp, tys);
    uint32_t P[4][4];
    float fs[4], ft[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
      int x0, x1, y0, y1;
      cell(sx + shx[k], a.W, x0, x1, fs[k]);
      cell(ty + shy[k], a.H, y0, y1, ft[k]);
      const int FW = FBX[k] * B, FH = FBY[k] * B;
      const int lx0 = min(max(x0 - fbx0[k] * B, 0), FW - 1), lx1 = min(max(x1 - fbx0[k] * B, 0), FW - 1);
      const int ly0 = min(max(y0 - fby0[k] * B, 0), FH - 1), ly1 = min(max(y1 - fby0[k] * B, 0), FH - 1);
      // word of footprint pixel (lx, ly) within the view's part of the tile
      const uint32_t *img = acc + k * FBM * SLOT;
      P[k][0] = img[((ly0 / B) * FBX[k] + lx0 / B) * SLOT + (ly0 % B) * B + lx0 % B];
      P[k][1] = img[((ly0 / B) * FBX[k] + lx1 / B) * SLOT + (ly0 % B) * B + lx1 % B];
      P[k][2] = img[((ly1 / B) * FBX[k] + lx0 / B) * SLOT + (ly1 % B) * B + lx0 % B];
      P[k][3] = img[((ly1 / B) * FBX[k] + lx1 / B) * SLOT + (ly1 % B) * B + lx1 % B];
    }
    interp_store(P, fs, ft, fu, fv, outn + (size_t)Yp * a.wo + X, plane);
  }
}

template <int B, bool FOCAL>
__global__ __launch_bounds__(kRenderThreads) void k_render(RenderArgs a) {
  extern __shared__ uint32_t smem[];
  const int n = blockIdx.z;
  render_tile<B, FOCAL>(a, a.views[n], a.out + (size_t)n * 3 * a.ho * a.wo, blockIdx.x, blockIdx.y, smem);
}

// Many render requests in one launch, possibly of different light fields and
// output sizes: workgroup (x, r) renders tile x of request r, and exits when
// the request has fewer tiles.
struct RenderReq {
  RenderArgs a;        // the request's light field, output size, tiling and output (views unused)
  lfc_view view;
  int ntx, ntiles;     // tile columns, tiles
};

template <int B>
__global__ __launch_bounds__(kRenderThreads) void k_render_multi(const RenderReq *reqs) {
  extern __shared__ uint32_t smem[];
  // one read of the record, at the start: every wave then works from the
  // same copy, however late it uses a field
  const RenderReq r = reqs[blockIdx.y];
  const int t = blockIdx.x;
  if (t >= r.ntiles) return;
  render_tile<B, false>(r.a, r.view, r.a.out, t % r.ntx, t / r.ntx, smem);
}

// ---------------------------------------------------------------------------
// whole light field as 8-bit RGB (the decode-then-interpolate render's input)
// ---------------------------------------------------------------------------

// LDS words before the tile: LUT; the start words of the strip's 3 x 64/B
// groups; a flag and a bit per node of the chunk for the views a render
// reads; the view mask; the chunk's per-node masks and first slots (a chunk
// has at most lfc::kRGBNodeCap nodes).
using lfc::kRGBNodeCap;
constexpr int kRGBNeedWords = 128;        // views a render may mask: at most 32 x 128
constexpr int kRGBHeadWords = 192 + 96 + 4 + kRGBNodeCap / 32 + kRGBNeedWords + 3 * kRGBNodeCap +
                               3 * kRGBNodeCap / 2 + 3 * kRGBNodeCap + 4 * kRGBNodeCap / 2;
constexpr int kRGBKeyWordsMax = 6144;     // key-view rows of a strip staged in LDS up to 24 KB

struct RGBArgs {
  const int16_t *rkv;
  const uint32_t *off;
  const uint32_t *srv;
  const uint32_t *sched;      // colour decode schedule: one record per strip (build_schedule_rgb on the host)
  const uint32_t *strip_off;  // [n_strips+1]
  const uint32_t *order;      // [n_strips] strip of each workgroup, costliest first
  const int32_t *batch;       // [nbatch][kBatchWords] runs of sibling leaves
  const uint32_t *vneed;      // [ceil(nv/32)] bit per view to write (nv <= 32 kRGBNeedWords), or null: every view
  uint32_t *out;              // [nv][hp][wp] pixels R | G << 8 | B << 16
  int nbx, nsx, L, q, wp, hp, nb, nbatch, nv;
  int n_top, key_words;       // LDS words of the strip's key-view rows of all channels (0: read from global)
  int tile_cap;
  int parts;                  // workgroups per strip: part p takes the chunks ci with ci % parts == p
  // with vneed null: the cameras of a render, whose four grid neighbours
  // each workgroup marks itself (null: every view, unless vneed is given)
  const lfc_view *views = nullptr;
  int nviews = 0, U = 0, V = 0;
};

// One workgroup = one strip of 64/B blocks of one block row, all three
// channels, or every parts-th chunk of it (a strip of three channels holds
// three times the blocks of a one-channel strip, so strips alone would not
// fill the chip).  Phase A stages the LUT, the strip's group starts, the
// view mask and the key-view rows; the groups and the decode schedule are
// read from global memory.  Per chunk of the strip's runs: its node masks
// and first slots are copied to LDS while (3) every stored residual block of
// the chunk, of any channel (with a view mask: of a node that a wanted view
// reads), is decoded once into the compact tile; then (4) one run per wave:
// a lane owns one sibling and 4 pixels of the strip's rows, sums key row +
// ancestor rows + leaf row of each channel, converts the pixels to RGB
// (inverse YCoCg-R, clamped) and stores 16 bytes per row.
// The work of one workgroup (strip st, part) of the colour kernel; the LUT
// in the first 192 words of smem is already filled.
template <int B, bool KEYS>
__device__ __forceinline__ void rgb_strip(const RGBArgs &a, int st, int part, uint32_t *smem) {
  constexpr int S = B * B, NBLK = 64 / B, H = B / 2, HR = B;   // HR rows per lane
  const uint16_t *lut = reinterpret_cast<const uint16_t *>(smem);   // 384 x u16 = 192 words
  uint32_t *s_o0 = smem + 192;                          // [3][NBLK] group start words
  uint32_t *s_nlist = smem + 288;                       // [0] listed pairs of the chunk ([2] is the multi kernel's)
  uint32_t *s_node = s_nlist + 4;                       // wanted nodes of the chunk, a bit each
  uint32_t *s_need = s_node + kRGBNodeCap / 32;         // the view mask
  uint32_t *s_mf = s_need + kRGBNeedWords;              // masks[3][nn], first slots (16-bit), run node positions[nq][3]
  uint16_t *s_list = reinterpret_cast<uint16_t *>(s_mf + 3 * kRGBNodeCap + 3 * kRGBNodeCap / 2 + 3 * kRGBNodeCap);
                                                        // (run << 2 | sibling) pairs of the chunk
  uint32_t *tile = smem + kRGBHeadWords;                // [tile_cap + 1][S/2], the last slot zero
  uint32_t *keys = tile + lf_tile_words(a.tile_cap, S); // [3][n_top][NBLK][S/2], blocks as in the tile
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int sx = st % a.nsx, by = st / a.nsx;
  const bool masked = a.vneed != nullptr || a.views != nullptr;
  if (tid < S / 2) tile[a.tile_cap * (S / 2) + tid] = 0u;
  if (tid < 64)
    for (int k = lane; k < 3 * NBLK; k += 64) {
      const int c = k / NBLK, bx = sx * NBLK + k % NBLK;
      s_o0[k] = bx < a.nbx ? a.off[3 * (by * a.nbx + bx) + c] : 0u;
    }
  if (a.vneed) {
    for (int w = tid; w < (a.nv + 31) / 32; w += kLFThreads) s_need[w] = a.vneed[w];
  } else if (a.views) {
    // the source views the cameras read: each camera's four grid neighbours
    for (int w = tid; w < (a.nv + 31) / 32; w += kLFThreads) s_need[w] = 0u;
    lds_barrier();
    for (int i = tid; i < a.nviews; i += kLFThreads) {
      int iu0, iu1, jv0, jv1;
      float fu, fv;
      cell(a.views[i].u, a.U, iu0, iu1, fu);
      cell(a.views[i].v, a.V, jv0, jv1, fv);
      const int vs[4] = {jv0 * a.U + iu0, jv0 * a.U + iu1, jv1 * a.U + iu0, jv1 * a.U + iu1};
#pragma unroll
      for (int k = 0; k < 4; k++) atomicOr(&s_need[vs[k] >> 5], 1u << (vs[k] & 31));
    }
  }
  if constexpr (KEYS) {
    const uint32_t *rk = reinterpret_cast<const uint32_t *>(a.rkv);
    for (int t0 = wave * 64; t0 < a.key_words; t0 += kLFThreads) {
      const int t = t0 + lane, wd = t % (S / 2), j = (t / (S / 2)) % NBLK;
      const int r = (t / (S / 2 * NBLK)) % a.n_top, c = t / (S / 2 * NBLK * a.n_top);
      const int bx = sx * NBLK + j;
      if (t < a.key_words && bx < a.nbx)
        __builtin_amdgcn_global_load_lds(
            (const __attribute__((address_space(1))) void *)(rk + ((size_t)(r * a.nb + by * a.nbx + bx) * 3 + c) *
                                                                  (S / 2) + wd),
            (__attribute__((address_space(3))) void *)(keys + t0), 4, 0, 0);
    }
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();

  // gather lane mapping: listed pair lane / 16, 4-pixel segment jseg (word pairs pp = 2 jseg,
  // 2 jseg + 1 of the strip's 32-word rows); the block and the word inside its row of each pair
  const int jseg = lane & 15;
  int jb[2], wib[2];
#pragma unroll
  for (int w = 0; w < 2; w++) {
    const int pp = 2 * jseg + w;
    jb[w] = (2 * pp) / B;
    wib[w] = ((2 * pp) % B) / 2;
  }
  const int px0 = sx * 64 + 4 * jseg;                   // first pixel of the segment
  const bool seg_in = sx * NBLK + jb[0] < a.nbx;        // the segment's first block is inside the image
  const bool wide = seg_in && (a.wp % 4 == 0);          // all 4 pixels inside, 16-byte aligned
  const uint32_t zslot = (uint32_t)a.tile_cap;
  const uint32_t vplane = (uint32_t)a.hp * (uint32_t)a.wp;
  auto wanted_view = [&](int vi) { return !masked || ((s_need[vi >> 5] >> (vi & 31)) & 1u); };
  const uint32_t *gs = a.sched + a.strip_off[st];
  const int nck = __builtin_amdgcn_readfirstlane((int)gs[0]);
  for (int ci = part; ci < nck; ci += a.parts) {
    const uint32_t *chunk = gs + gs[1 + ci];
    const uniform_i32 sch = as_uniform(reinterpret_cast<const int32_t *>(chunk));
    const int q0 = sch[0], nq = sch[1], nn = sch[2];
    const uint32_t n0 = (uint32_t)sch[3], n01 = (uint32_t)sch[4], n = (uint32_t)sch[5];
    const int mf_words = 3 * nn + (3 * nn + 1) / 2;
    const uniform_i32 runs = sch + 6 + mf_words;
    const uint32_t *ents = chunk + 6 + mf_words + 3 * nq;
    const uint32_t *items = ents + n;
    // with a view mask, the chunk's (run, sibling) pairs of wanted views are
    // listed in LDS and the nodes they read are marked (a chunk with none is
    // skipped whole); without one, pair e is sibling e % 4 of run e / 4
    int n_list = 4 * nq;
    if (masked) {
      for (int w = tid; w < kRGBNodeCap / 32; w += kLFThreads) s_node[w] = 0u;
      if (tid == 0) *s_nlist = 0u;
      // (barriers on LDS only: a full barrier would also wait for the stores
      // of the previous chunk's gather)
      lds_barrier();
      for (int qi = wave; qi < nq; qi += kLFWaves) {
        const uniform_i32 rec = as_uniform(a.batch + (size_t)(q0 + qi) * lfc::kBatchWords);
        const int nsib = rec[0];
        bool wanted[4];
#pragma unroll
        for (int k = 0; k < 4; k++) wanted[k] = k < nsib && wanted_view(max(rec[1 + k], 0));
        if (!(wanted[0] || wanted[1] || wanted[2] || wanted[3])) continue;
        const bool mine = lane == 0 ? wanted[0] : (lane == 1 ? wanted[1] : (lane == 2 ? wanted[2] : wanted[3]));
        if (lane < 4 && mine) s_list[atomicAdd(s_nlist, 1u)] = (uint16_t)(qi << 2 | lane);
        const uint32_t w0 = (uint32_t)runs[3 * qi], w1 = (uint32_t)runs[3 * qi + 1], w2 = (uint32_t)runs[3 * qi + 2];
        const int anc_ln[4] = {(int)(w0 >> 16), (int)(w1 & 0xFFFFu), (int)(w1 >> 16), (int)(w2 & 0xFFFFu)};
        int ln = -1;
        if (lane < 4 && a.L > 1 && mine)
          ln = (int)(w0 & 0xFFFFu) + lane;
        else if (lane >= 4 && lane < 8 && lane - 4 < a.L - 2)
          ln = lane == 4 ? anc_ln[0] : (lane == 5 ? anc_ln[1] : (lane == 6 ? anc_ln[2] : anc_ln[3]));
        if (ln >= 0) atomicOr(&s_node[ln >> 5], 1u << (ln & 31));
      }
      lds_barrier();
      n_list = __builtin_amdgcn_readfirstlane((int)*s_nlist);
      if (n_list == 0) {
        lds_barrier();   // every wave has read the count before the next chunk clears it
        continue;
      }
    }
    // the chunk's node masks, first slots and run records into LDS, in
    // flight during the decode (the gather then reads no global memory but
    // the run's view list)
    const int tab_words = mf_words + 3 * nq;
    for (int w0 = wave * 64; w0 < tab_words; w0 += kLFThreads)
      if (w0 + lane < tab_words)
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)(chunk + 6 + w0 + lane),
                                         (__attribute__((address_space(3))) void *)(s_mf + w0), 4, 0, 0);
    // (3) decode every stored block of the chunk (that a wanted view reads) into its tile slot
    uint32_t e_nx = 0, t_nx = 0;   // the lane's next entry, requested ahead (as in the one-channel kernel)
    if ((uint32_t)tid < n) {
      e_nx = ents[tid];
      t_nx = items[tid];
    }
    for (uint32_t it = tid; it < n; it += kLFThreads) {
      const uint32_t e = e_nx, t = t_nx;
      if (it + kLFThreads < n) {
        e_nx = ents[it + kLFThreads];
        t_nx = items[it + kLFThreads];
      }
      if (masked) {
        const uint32_t ln = (t >> 8) & 4095u;
        if (!((s_node[ln >> 5] >> (ln & 31u)) & 1u)) continue;
      }
      const uint32_t *gw = a.srv + s_o0[((t >> 6) & 3u) * NBLK + (t & 63u)];
      uint32_t d[S / 2];
      if (it < n0) decode_block_k<B, 0>(gw, e, a.q, lut, d);
      else if (it < n01) decode_block_k<B, 1>(gw, e, a.q, lut, d);
      else decode_block_k<B, 2>(gw, e, a.q, lut, d);
      uint32_t *dst = tile + (t >> 20) * (S / 2);
      if constexpr (S / 2 >= 4) {
#pragma unroll
        for (int w = 0; w < S / 2; w += 4)
          *reinterpret_cast<uint4 *>(dst + w) = make_uint4(d[w], d[w + 1], d[w + 2], d[w + 3]);
      } else {
        *reinterpret_cast<uint2 *>(dst) = make_uint2(d[0], d[1]);
      }
    }
    __builtin_amdgcn_s_waitcnt(0x0f70);   // vmcnt(0): this wave's copies of the node table have landed
    lds_barrier();
    const uint16_t *firsts = reinterpret_cast<const uint16_t *>(s_mf + 3 * nn);
    const uint32_t *s_runs = s_mf + mf_words;
    // (4) four listed (run, sibling) pairs per wave at a time, one per
    // 16-lane group; each pair's view and key view come through the scalar
    // unit (no vector load, which would wait for the wave's stores)
    for (int e0 = wave * 4; e0 < n_list; e0 += 4 * kLFWaves) {
      constexpr int y0 = 0;
      uint32_t ens[4];
      if (masked) {
        const uint2 pr = *reinterpret_cast<const uint2 *>(s_list + e0);
        ens[0] = pr.x & 0xFFFFu;
        ens[1] = pr.x >> 16;
        ens[2] = pr.y & 0xFFFFu;
        ens[3] = pr.y >> 16;
      } else {
#pragma unroll
        for (int g = 0; g < 4; g++) ens[g] = (uint32_t)(e0 + g);
      }
      int f_vi[4], f_root[4], f_q[4], f_so[4], f_ok[4];
#pragma unroll
      for (int g = 0; g < 4; g++) {
        const int en = e0 + g < n_list ? __builtin_amdgcn_readfirstlane((int)ens[g]) : 0;
        f_q[g] = en >> 2;
        f_so[g] = en & 3;
        const uniform_i32 rec = as_uniform(a.batch + (size_t)(q0 + f_q[g]) * lfc::kBatchWords);
        f_vi[g] = rec[1 + f_so[g]];
        f_root[g] = rec[5];
        f_ok[g] = e0 + g < n_list && f_so[g] < rec[0];   // (listed pairs are always present siblings)
      }
      const int grp = lane >> 4;
      auto pick = [&](const int (&f)[4]) { return grp == 0 ? f[0] : (grp == 1 ? f[1] : (grp == 2 ? f[2] : f[3])); };
      const int vi = pick(f_vi), root = pick(f_root), qi = pick(f_q), so = pick(f_so);
      const bool live = seg_in && pick(f_ok);
      const uint32_t w0 = s_runs[3 * qi], w1 = s_runs[3 * qi + 1], w2 = s_runs[3 * qi + 2];
      const int anc_ln[4] = {(int)(w0 >> 16), (int)(w1 & 0xFFFFu), (int)(w1 >> 16), (int)(w2 & 0xFFFFu)};
      const int leaf = min((int)(w0 & 0xFFFFu) + so, max(nn - 1, 0));   // the lane's own leaf
      uint32_t x[3][HR][2];
      // the lane's words of a block slot (tile or key rows, same layout):
      // B = 4, the whole 4 x 4 block in two 16-byte reads; B = 2, both rows
      // of each of its two blocks in one 8-byte read; B = 8, half of each row
      auto read_slot = [&](const uint32_t *slot0, const uint32_t *slot1, bool add, uint32_t (&xc)[HR][2]) {
        if constexpr (B == 4) {
          const uint4 v0 = *reinterpret_cast<const uint4 *>(slot0), v1 = *reinterpret_cast<const uint4 *>(slot0 + 4);
          const uint32_t w[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
#pragma unroll
          for (int y = 0; y < 4; y++)
#pragma unroll
            for (int k = 0; k < 2; k++) xc[y][k] = add ? add_pk(xc[y][k], w[2 * y + k]) : w[2 * y + k];
        } else if constexpr (B == 2) {
          const uint2 v0 = *reinterpret_cast<const uint2 *>(slot0), v1 = *reinterpret_cast<const uint2 *>(slot1);
          const uint32_t w[2][2] = {{v0.x, v1.x}, {v0.y, v1.y}};
#pragma unroll
          for (int y = 0; y < 2; y++)
#pragma unroll
            for (int k = 0; k < 2; k++) xc[y][k] = add ? add_pk(xc[y][k], w[y][k]) : w[y][k];
        } else {
#pragma unroll
          for (int y = 0; y < HR; y++) {
            const uint2 v = *reinterpret_cast<const uint2 *>(slot0 + y * H + wib[0]);
            xc[y][0] = add ? add_pk(xc[y][0], v.x) : v.x;
            xc[y][1] = add ? add_pk(xc[y][1], v.y) : v.y;
          }
        }
      };
#pragma unroll
      for (int c = 0; c < 3; c++) {
        // key-view rows
        if constexpr (KEYS) {
          const uint32_t *kb = keys + (c * a.n_top + root) * (NBLK * (S / 2));
          read_slot(kb + jb[0] * (S / 2), kb + jb[1] * (S / 2), false, x[c]);
        } else {
#pragma unroll
          for (int y = 0; y < HR; y++) {
#pragma unroll
            for (int w = 0; w < 2; w++) {
              const int bx = sx * NBLK + jb[w];
              x[c][y][w] = bx < a.nbx ? reinterpret_cast<const uint32_t *>(
                                            a.rkv)[((size_t)(root * a.nb + by * a.nbx + bx) * 3 + c) * (S / 2) +
                                                   (y0 + y) * H + wib[w]]
                                      : 0u;
            }
          }
        }
        // rows of node ln added
        auto add_node = [&](int ln) {
          const uint32_t mk = s_mf[c * nn + ln], f = firsts[c * nn + ln];
          auto slot = [&](int w) {
            const uint32_t j = (uint32_t)jb[w];
            const uint32_t sl = ((mk >> j) & 1u) ? f + (uint32_t)__popc(mk & ((1u << j) - 1u)) : zslot;
            return tile + sl * (S / 2);
          };
          read_slot(slot(0), B == 2 ? slot(1) : nullptr, true, x[c]);
        };
#pragma unroll
        for (int k = 0; k < 4; k++)
          if (k < a.L - 2) add_node(anc_ln[k]);
        if (a.L > 1) add_node(leaf);
      }
      if (!live) continue;
      uint32_t *dst = a.out + (uint32_t)vi * vplane + (uint32_t)(by * B + y0) * (uint32_t)a.wp + (uint32_t)px0;
#pragma unroll
      for (int y = 0; y < HR; y++) {
        uint32_t p[4];
#pragma unroll
        for (int w = 0; w < 2; w++) {
          p[2 * w] = rgb_pack(lo16(x[0][y][w]), lo16(x[1][y][w]), lo16(x[2][y][w]));
          p[2 * w + 1] = rgb_pack(hi16(x[0][y][w]), hi16(x[1][y][w]), hi16(x[2][y][w]));
        }
        uint32_t *row = dst + (uint32_t)y * (uint32_t)a.wp;
        if (wide) {
          *reinterpret_cast<uint4 *>(row) = make_uint4(p[0], p[1], p[2], p[3]);
        } else {
#pragma unroll
          for (int k = 0; k < 4; k++)
            if (px0 + k < a.wp) row[k] = p[k];
        }
      }
    }
    lds_barrier();
  }
}

template <int B, bool KEYS>
__global__ __launch_bounds__(kLFThreads) void k_decode_rgb(RGBArgs a) {
  extern __shared__ uint32_t smem[];
  uint16_t *lut = reinterpret_cast<uint16_t *>(smem);
  for (int t = threadIdx.x; t < kLutEntries; t += kLFThreads) lut[t] = lut_entry(t);
  rgb_strip<B, KEYS>(a, (int)a.order[blockIdx.x / a.parts], blockIdx.x % a.parts, smem);
}

// The colour decode of several light fields in one persistent launch: the
// work items are every light field's (strip, part) pairs, each light field's
// strips costliest first; workgroups stay resident and take the next item
// from a device counter until none is left.  The last workgroup to finish
// puts the counters back to zero, so the next launch (or graph replay) needs
// no clearing; launches that share counters must not overlap.
struct RGBMultiArgs {
  const RGBArgs *lfs;      // [n_lf], every one of block size B
  const int32_t *first;    // [n_lf + 1] first work item of each light field (items = strips x parts)
  int n_lf, n_items;
  uint32_t *ctr;           // [2]: next work item, finished workgroups
};

template <int B, bool KEYS>
__global__ __launch_bounds__(kLFThreads) void k_decode_rgb_multi(RGBMultiArgs m) {
  extern __shared__ uint32_t smem[];
  uint16_t *lut = reinterpret_cast<uint16_t *>(smem);
  uint32_t *s_item = smem + 288 + 2;   // a free word of the chunk flags
  for (int t = threadIdx.x; t < kLutEntries; t += kLFThreads) lut[t] = lut_entry(t);
  const uniform_i32 first = as_uniform(m.first);
  for (;;) {
    lds_barrier();   // every wave is done with the previous item's LDS (its stores may still be in flight)
    if (threadIdx.x == 0) *s_item = atomicAdd(&m.ctr[0], 1u);
    lds_barrier();
    const int item = __builtin_amdgcn_readfirstlane((int)*s_item);
    if (item >= m.n_items) break;
    int lf = 0;
    while (lf + 1 < m.n_lf && first[lf + 1] <= item) lf++;
    const RGBArgs a = m.lfs[lf];
    const int local = item - first[lf];
    rgb_strip<B, KEYS>(a, (int)a.order[local / a.parts], local % a.parts, smem);
  }
  if (threadIdx.x == 0) {
    __threadfence();
    if (atomicAdd(&m.ctr[1], 1u) == gridDim.x - 1) {
      atomicExch(&m.ctr[0], 0u);
      atomicExch(&m.ctr[1], 0u);
    }
  }
}

// Novel views from fully decoded 8-bit RGB source views ([nv][hp][wp]): one
// thread per output pixel, its 16 taps one word each, the same lerps as
// render_tile.  Used when a batch of views needs about as many source blocks
// as the whole light field holds.
struct InterpRGBArgs {
  const uint32_t *rgb;
  uint32_t rgb_bytes;   // bytes of the decoded views (below 4 GiB)
  const lfc_view *views;
  float *out;
  int wo, ho, U, V, W, H, wp, hp;
  float disp;       // focal disparity (as RenderArgs)
  float sxs, tys;   // W / wo and H / ho, rounded once on the host as the other renderers round them
};

// Output pixel (X, Yp) of view vw into o (its view's [3][ho][wo] planes).
template <bool FOCAL>
__device__ __forceinline__ void interp_rgb_pixel(const InterpRGBArgs &a, const lfc_view &vw, float *o, int X,
                                                 int Yp) {
  int iu0, iu1, jv0, jv1, x0, x1, y0, y1;
  float fu, fv;
  cell(vw.u, a.U, iu0, iu1, fu);
  cell(vw.v, a.V, jv0, jv1, fv);
  const float sx = src_pos(vw.s, X, a.sxs), ty = src_pos(vw.t, Yp, a.tys);
  // taps through a buffer resource: 32-bit byte offsets from one base (the
  // decoded views take less than 4 GiB)
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<uint32_t *>(a.rgb), 0, a.rgb_bytes, 0x00020000);
  const uint32_t vbytes = 4u * (uint32_t)a.hp * (uint32_t)a.wp, rbytes = 4u * (uint32_t)a.wp;
  const uint32_t vis[4] = {(uint32_t)(jv0 * a.U + iu0), (uint32_t)(jv0 * a.U + iu1), (uint32_t)(jv1 * a.U + iu0),
                           (uint32_t)(jv1 * a.U + iu1)};
  uint32_t P[4][4];
  float fs[4], ft[4];
#pragma unroll
  for (int k = 0; k < 4; k++) {
    cell(sx + focal_shift<FOCAL>(a.disp, vw.u, a.U, (k & 1) ? iu1 : iu0), a.W, x0, x1, fs[k]);
    cell(ty + focal_shift<FOCAL>(a.disp, vw.v, a.V, (k & 2) ? jv1 : jv0), a.H, y0, y1, ft[k]);
    // a row's offset goes in the load's scalar offset, the column in the
    // per-lane one, and the hardware adds them
    if constexpr (FOCAL) {   // (the shifted row is computed per lane otherwise)
      y0 = __builtin_amdgcn_readfirstlane(y0);
      y1 = __builtin_amdgcn_readfirstlane(y1);
    }
    const uint32_t r0 = __builtin_amdgcn_readfirstlane(vis[k] * vbytes + (uint32_t)y0 * rbytes);
    const uint32_t r1 = __builtin_amdgcn_readfirstlane(vis[k] * vbytes + (uint32_t)y1 * rbytes);
    const uint32_t c0 = 4u * (uint32_t)x0, c1 = 4u * (uint32_t)x1;
    P[k][0] = __builtin_amdgcn_raw_buffer_load_b32(rs, c0, r0, 0);
    P[k][1] = __builtin_amdgcn_raw_buffer_load_b32(rs, c1, r0, 0);
    P[k][2] = __builtin_amdgcn_raw_buffer_load_b32(rs, c0, r1, 0);
    P[k][3] = __builtin_amdgcn_raw_buffer_load_b32(rs, c1, r1, 0);
  }
  interp_store(P, fs, ft, fu, fv, o + (size_t)Yp * a.wo + X, (size_t)a.ho * a.wo);
}

template <bool FOCAL>
__global__ __launch_bounds__(kThreads) void k_interp_rgb(InterpRGBArgs a) {
  // grid (row pieces, view, row): the workgroups that run together render one
  // output row of every view, whose taps come from nearby rows of the same
  // few source views, so the caches serve those rows once for all views
  // (a grid that gave each of the eight dies its own band of rows measured
  // no faster)
  const int X = blockIdx.x * kThreads + threadIdx.x, n = blockIdx.y, Yp = blockIdx.z;
  if (X >= a.wo) return;
  interp_rgb_pixel<FOCAL>(a, a.views[n], a.out + (size_t)n * 3 * a.ho * a.wo, X, Yp);
}

// Requests of several light fields and output sizes interpolated in one
// launch: workgroup (piece, request, row) exits when the request's output is
// smaller.  A request's record carries its light field's decoded views
// (views unused; the camera is in the record).
struct InterpReq {
  InterpRGBArgs a;
  lfc_view view;
};

__global__ __launch_bounds__(kThreads) void k_interp_multi(const InterpReq *reqs) {
  const InterpReq r = reqs[blockIdx.y];
  const int X = blockIdx.x * kThreads + threadIdx.x, Yp = blockIdx.z;
  if (X >= r.a.wo || Yp >= r.a.ho) return;
  interp_rgb_pixel<false>(r.a, r.view, r.a.out, X, Yp);
}

// ---------------------------------------------------------------------------
// host-side checks and launches
// ---------------------------------------------------------------------------

using lfc::fail;

lfc_status check_device(const lfc_lf *lf, const char *who) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(LFC_E_HIP, std::string(who) + ": no current device");
  if (dev != lf->device)
    return fail(LFC_E_INVALID, std::string(who) + ": the current device is not the one the light field was opened on");
  return LFC_OK;
}

// the device buffer at p must hold at least need bytes inside one allocation
lfc_status check_buffer(const void *p, size_t need, size_t align, const char *who, const char *what) {
  if (!p) return fail(LFC_E_INVALID, std::string(who) + ": null " + what);
  if (reinterpret_cast<uintptr_t>(p) % align)
    return fail(LFC_E_INVALID, std::string(who) + ": " + what + " is not " + std::to_string(align) + "-byte aligned");
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, const_cast<void *>(p)) != hipSuccess || !base) {
    (void)hipGetLastError();
    return fail(LFC_E_INVALID, std::string(who) + ": " + what + " is not device memory");
  }
  const size_t off = static_cast<const char *>(p) - static_cast<const char *>(base);
  if (off + need > size) return fail(LFC_E_INVALID, std::string(who) + ": " + what + " is too small");
  return LFC_OK;
}

RAArgs ra_args(const lfc_lf *lf) {
  const lfc::Geometry &g = lf->geo;
  return RAArgs{lf->d_rkv, lf->d_off, lf->d_srv, lf->d_dbase, lf->d_poff, lf->d_path, lf->d_root,
                g.nb, g.nbx, g.nv(), g.nbw, g.L, g.q, lf->d_dir2};
}

lfc_status launched(const char *who) {
  const hipError_t he = hipGetLastError();
  if (he != hipSuccess) return fail(LFC_E_HIP, std::string(who) + ": launch failed: " + hipGetErrorString(he));
  return LFC_OK;
}

// LDS a workgroup may use on the current device (queried once per device).
int max_lds_bytes() {
  constexpr int kDevices = 64;
  static std::atomic<int> cached[kDevices];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return 64 * 1024;
  if (dev < kDevices)
    if (const int v = cached[dev].load(std::memory_order_relaxed)) return v;
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0) {
    (void)hipGetLastError();
    v = 64 * 1024;
  }
  if (dev < kDevices) cached[dev].store(v, std::memory_order_relaxed);
  return v;
}

// Compute units of the current device (queried once per device).
int device_cus() {
  constexpr int kDevices = 64;
  static std::atomic<int> cached[kDevices];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return 256;
  if (dev < kDevices)
    if (const int v = cached[dev].load(std::memory_order_relaxed)) return v;
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) {
    (void)hipGetLastError();
    v = 256;
  }
  if (dev < kDevices) cached[dev].store(v, std::memory_order_relaxed);
  return v;
}

// Stream-ordered scratch from a memory pool of the library's own per device,
// which keeps up to 1 GiB of freed memory for the next call instead of
// returning it at each synchronisation (the default pool's release threshold
// is zero); the process's default pool is left as it is.
hipMemPool_t scratch_pool() {
  constexpr int kDevices = 64;
  static std::mutex mu;
  static hipMemPool_t pools[kDevices] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kDevices) return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  if (!pools[dev]) {
    hipMemPoolProps props{};
    props.allocType = hipMemAllocationTypePinned;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = dev;
    hipMemPool_t pl = nullptr;
    if (hipMemPoolCreate(&pl, &props) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    uint64_t keep = (uint64_t)1 << 30;
    if (hipMemPoolSetAttribute(pl, hipMemPoolAttrReleaseThreshold, &keep) != hipSuccess) (void)hipGetLastError();
    pools[dev] = pl;
  }
  return pools[dev];
}

// LDS of the whole-field kernel: the fixed part (LUT and extents, residual
// tile, key-view rows) plus staging for the strip's groups and decode
// schedule, up to 80 KB so that two workgroups share a compute unit.
// Output larger than this (the MI355X's 256 MiB Infinity Cache) cannot stay
// cached for a consumer, and stored normally it would evict the compressed
// input; it is stored with the non-temporal hint.
constexpr uint64_t kStreamOutBytes = (uint64_t)256 << 20;

// stage_cap < 0: as much LDS staging as the strips need, up to the 80 KB
// workgroup budget; else at most stage_cap words (tests of the tiers).
template <int B>
lfc_status decode_images(const lfc_lf *lf, int16_t *out, hipStream_t s, int64_t stage_cap = -1) {
  const lfc::Geometry &g = lf->geo;
  constexpr int NBLK = 64 / B;

  // key-view rows of a strip, when they take at most 16 KB
  const int64_t key_words = (int64_t)g.n_top * NBLK * (B * B / 2) <= 4096 ? (int64_t)g.n_top * NBLK * (B * B / 2) : 0;
  if ((int64_t)3 * g.hp * g.wp >= ((int64_t)1 << 32))
    return fail(LFC_E_UNSUPPORTED, "lfc_decode_blocks: view too large for the whole-field kernel");
  const int64_t fixed = kLFHeadWords + (int64_t)lf_tile_words(lf->tile_cap, B * B) + key_words + lfc::kLFTabWords;
  const int64_t limit = max_lds_bytes() / 4;
  if (fixed > limit)
    return fail(LFC_E_UNSUPPORTED, "lfc_decode_blocks: tree too large for the whole-field kernel; use BLOCKS layout");
  const int64_t target = std::min<int64_t>(limit, std::max<int64_t>(80 * 1024 / 4, fixed));
  int64_t cap = std::min<int64_t>(target - fixed, (int64_t)lf->max_strip_words + kStagePad);
  if (stage_cap >= 0) cap = std::min<int64_t>(cap, stage_cap);
  const size_t lds = 4 * (size_t)(fixed + cap);
  LFArgs a{lf->d_rkv, lf->d_off, lf->d_srv, lf->d_sched, lf->d_strip_off, lf->d_order, lf->d_batch, out,
           g.nbx, g.nv(), g.L, g.q, g.wp, g.hp, g.nb, lf->n_batch, (int)cap,
           (int)(g.wp % 8 == 0 && reinterpret_cast<uintptr_t>(out) % 16 == 0), g.n_top, (int)key_words,
           lf->tile_cap, (int)((uint64_t)g.nv() * 3 * g.hp * g.wp * 2 > kStreamOutBytes)};
  dim3 grid((g.nbx + NBLK - 1) / NBLK, g.nby, 3);
  hipLaunchKernelGGL(k_decode_lf<B>, grid, dim3(kLFThreads), lds, s, a);
  return launched("lfc_decode_blocks");
}

// Every view (or those whose bit is set in vneed) as 8-bit RGB words
// [nv][hp][wp], inverse YCoCg-R and clamp applied to the decoded samples.
template <int B>
lfc_status decode_rgb(const lfc_lf *lf, uint32_t *out, const uint32_t *vneed, hipStream_t s, const char *who,
                      const lfc_view *views = nullptr, int nviews = 0) {
  const lfc::Geometry &g = lf->geo;
  constexpr int NBLK = 64 / B;
  if ((uint64_t)g.nv() * g.hp * g.wp >= ((uint64_t)1 << 32))
    return fail(LFC_E_UNSUPPORTED, std::string(who) + ": light field too large for 32-bit pixel indices");
  const int64_t kw = (int64_t)3 * g.n_top * B * 32;
  const int key_words = kw <= kRGBKeyWordsMax ? (int)kw : 0;
  const size_t lds = 4 * ((size_t)kRGBHeadWords + (size_t)lf_tile_words(lf->tile_cap_rgb, B * B) + (size_t)key_words);
  if (lds > (size_t)max_lds_bytes())
    return fail(LFC_E_UNSUPPORTED, std::string(who) + ": tree too large for the colour whole-field kernel");
  const int nsx = (g.nbx + NBLK - 1) / NBLK, nstrips = g.nby * nsx;
  // workgroups per strip: enough for several rounds of the resident
  // workgroups (about three per compute unit), at most the strips' chunk count
  int parts = std::max(1, std::min(lf->rgb_max_chunks, (3 * 3 * device_cus() + nstrips - 1) / nstrips));
  // a view mask longer than the kernel's LDS copy of it: every view is decoded
  if (g.nv() > 32 * kRGBNeedWords) vneed = nullptr, views = nullptr;
  RGBArgs a{lf->d_rkv, lf->d_off, lf->d_srv, lf->d_sched_rgb, lf->d_strip_off_rgb, lf->d_order_rgb, lf->d_batch,
            vneed, out, g.nbx, nsx, g.L, g.q, g.wp, g.hp, g.nb, lf->n_batch, g.nv(), g.n_top, key_words,
            lf->tile_cap_rgb, parts};
  if (!vneed && views && nviews > 0) {
    a.views = views;
    a.nviews = nviews;
    a.U = g.U;
    a.V = g.V;
  }
  const dim3 grid((unsigned)(nstrips * parts));
  if (key_words)
    hipLaunchKernelGGL((k_decode_rgb<B, true>), grid, dim3(kLFThreads), lds, s, a);
  else
    hipLaunchKernelGGL((k_decode_rgb<B, false>), grid, dim3(kLFThreads), lds, s, a);
  return launched(who);
}

template <int B>
lfc_status decode_list(const lfc_lf *lf, const int32_t *req, int64_t n, int16_t *out, hipStream_t s, int stop = 0) {
  constexpr int RPW = 64 / (3 * B);
  BlocksArgs a{ra_args(lf), req, out, lf->d_err, n, stop};
  const int64_t waves = (n + RPW - 1) / RPW;
  const int64_t blocks = (waves + kThreads / 64 - 1) / (kThreads / 64);
  if (blocks > 0x7FFFFFFF) return fail(LFC_E_INVALID, "lfc_decode_blocks: too many requests");
  hipLaunchKernelGGL(k_decode_blocks<B>, dim3((unsigned)blocks), dim3(kThreads), 0, s, a);
  return launched("lfc_decode_blocks");
}

// Tile of output pixels per workgroup, and the largest footprint (in blocks)
// any tile can need; starting from TX x TY, shrinks the tile (if allowed)
// until the footprint fits 64 KB of LDS.
struct RenderPlan {
  int TX, TY, fbx, fby;
  size_t lds;
};

bool plan_render(const lfc::Geometry &g, int wo, int ho, RenderPlan &pl, int TX = 64, int TY = 16,
                 bool shrink = true) {
  const double sxs = (double)g.W / wo, tys = (double)g.H / ho;
  for (;;) {
    // footprint span: (T-1)*scale pixels plus the 1-pixel widening on each
    // side, the interpolation neighbour and float slack, then block alignment
    // a tile never spans more than the output
    const int tw = std::min(TX, wo), th = std::min(TY, ho);
    const int fbx = ((int)std::ceil((tw - 1) * sxs) + 5 + g.B - 1) / g.B + 2;
    const int fby = ((int)std::ceil((th - 1) * tys) + 5 + g.B - 1) / g.B + 2;
    const size_t lds = 4 * ((size_t)kLutEntries / 2 + (size_t)4 * fbx * fby * (3 * g.B * g.B / 2));
    if (lds <= 64 * 1024) {
      pl = RenderPlan{TX, TY, fbx, fby, lds};
      return true;
    }
    if (!shrink) return false;
    if (TY > 2) TY /= 2;
    else if (TX > 8) TX /= 2;
    else return false;
  }
}

// Decoding every source view once and interpolating from the decoded planes
// pays off when the batch's footprints together cover about as many blocks as
// the light field holds: each output pixel reads four views, and the
// whole-field decode is several times cheaper per block than decoding tile
// footprints.  lfc_render_views_ex forces either path.
bool render_decoded(const lfc::Geometry &g, int32_t n, int32_t wo, int32_t ho) {
  return 20.0 * n * wo * ho >= (double)g.nv() * g.hp * g.wp;
}

// A render request resolved to one launch shape: decode-then-interpolate, or
// per-tile footprint decode with a tile plan.
struct RenderChoice {
  bool decoded;
  RenderPlan pl;
  float disp;   // focal disparity
};

// cfg NULL or path LFC_RENDER_AUTO: the library's choice (render_decoded, and
// the largest tile up to 64 x 16 whose footprint fits); LFC_RENDER_TILES with
// tile_w x tile_h (0: 64 x 16, shrunk to fit) or LFC_RENDER_DECODED.
lfc_status choose_render(const lfc_lf *lf, int32_t n, int32_t wo, int32_t ho, const lfc_render_config *cfg,
                         RenderChoice &rc, const char *who) {
  const lfc::Geometry &g = lf->geo;
  const int path = cfg ? cfg->path : LFC_RENDER_AUTO;
  if (path != LFC_RENDER_AUTO && path != LFC_RENDER_TILES && path != LFC_RENDER_DECODED)
    return fail(LFC_E_INVALID, std::string(who) + ": unknown render path");
  rc.disp = cfg ? cfg->disparity : 0.0f;
  if (!std::isfinite(rc.disp) || std::fabs(rc.disp) > 1.0e6f)
    return fail(LFC_E_INVALID, std::string(who) + ": disparity must be finite, |d| <= 1e6");
  // the decoded path addresses its scratch with 32-bit byte offsets
  const bool fits = (uint64_t)g.nv() * g.hp * g.wp * 4 < ((uint64_t)1 << 32);
  if (path == LFC_RENDER_DECODED && !fits)
    return fail(LFC_E_UNSUPPORTED, std::string(who) + ": the decoded views would take 4 GiB or more");
  rc.decoded = fits && (path == LFC_RENDER_AUTO ? render_decoded(g, n, wo, ho) : path == LFC_RENDER_DECODED);
  if (rc.decoded) return LFC_OK;
  int TX = 64, TY = 16;
  bool shrink = true;
  if (path == LFC_RENDER_TILES && (cfg->tile_w || cfg->tile_h)) {
    if (cfg->tile_w < 1 || cfg->tile_h < 1 || cfg->tile_w > 1024 || cfg->tile_h > 1024)
      return fail(LFC_E_INVALID, std::string(who) + ": tile_w and tile_h must be 1..1024 (or both 0)");
    TX = cfg->tile_w;
    TY = cfg->tile_h;
    shrink = false;
  }
  if (!plan_render(g, wo, ho, rc.pl, TX, TY, shrink))
    return fail(LFC_E_UNSUPPORTED, std::string(who) + (shrink ? ": output too strongly minified for the tile footprint"
                                                             : ": the tile's source footprint exceeds 64 KB of LDS"));
  return LFC_OK;
}

// Scratch of the decode-then-interpolate path: the source views as 8-bit
// RGB words.
size_t rgb_bytes(const lfc::Geometry &g) { return (size_t)g.nv() * g.hp * g.wp * sizeof(uint32_t); }
size_t decoded_bytes(const lfc::Geometry &g) { return rgb_bytes(g); }

// One render with a resolved choice.  The decoded path decodes into ws when
// given, else into stream-ordered scratch from the library's pool.
template <int B>
lfc_status render_with(const lfc_lf *lf, const lfc_view *views, int32_t n, int32_t wo, int32_t ho, float *out,
                       const RenderChoice &rc, void *ws, hipStream_t s) {
  const lfc::Geometry &g = lf->geo;
  if (rc.decoded) {
    void *dec = ws;
    if (!dec && lfc::scratch_alloc(&dec, decoded_bytes(g), s) != LFC_OK)
      return fail(LFC_E_NOMEM, "lfc_render_views: scratch for the decoded views");
    uint32_t *rgb = static_cast<uint32_t *>(dec);
    // the views the batch reads (found by each workgroup of the colour
    // decode from the cameras) decoded, then the interpolation
    lfc_status st = decode_rgb<B>(lf, rgb, nullptr, s, "lfc_render_views", views, n);
    if (st == LFC_OK) {
      InterpRGBArgs ia{rgb, (uint32_t)rgb_bytes(g), views, out, wo, ho, g.U, g.V, g.W, g.H, g.wp, g.hp, rc.disp,
                       (float)g.W / (float)wo, (float)g.H / (float)ho};
      const dim3 grid((wo + kThreads - 1) / kThreads, n, ho);
      if (rc.disp != 0.0f)
        hipLaunchKernelGGL(k_interp_rgb<true>, grid, dim3(kThreads), 0, s, ia);
      else
        hipLaunchKernelGGL(k_interp_rgb<false>, grid, dim3(kThreads), 0, s, ia);
      st = launched("lfc_render_views");
    }
    if (!ws && hipFreeAsync(dec, s) != hipSuccess && st == LFC_OK)
      st = fail(LFC_E_HIP, "lfc_render_views: scratch release");
    return st;
  }
  const RenderPlan &pl = rc.pl;
  RenderArgs a{ra_args(lf), views, out, wo, ho, g.U, g.V, g.W, g.H, pl.TX, pl.TY, pl.fbx, pl.fby, rc.disp};
  dim3 grid((wo + pl.TX - 1) / pl.TX, (ho + pl.TY - 1) / pl.TY, n);
  if (rc.disp != 0.0f)
    hipLaunchKernelGGL((k_render<B, true>), grid, dim3(kRenderThreads), pl.lds, s, a);
  else
    hipLaunchKernelGGL((k_render<B, false>), grid, dim3(kRenderThreads), pl.lds, s, a);
  return launched("lfc_render_views");
}

lfc_status render_any(const lfc_lf *lf, const lfc_view *views, int32_t n, int32_t wo, int32_t ho, float *out,
                      const RenderChoice &rc, void *ws, hipStream_t s) {
  switch (lf->geo.B) {
    case 2: return render_with<2>(lf, views, n, wo, ho, out, rc, ws, s);
    case 4: return render_with<4>(lf, views, n, wo, ho, out, rc, ws, s);
    default: return render_with<8>(lf, views, n, wo, ho, out, rc, ws, s);
  }
}

// Argument checks shared by the render entry points.
lfc_status check_render(const lfc_lf *lf, const lfc_view *d_views, int32_t n, int32_t out_w, int32_t out_h,
                        const float *d_out, const char *who) {
  if (!lf) return fail(LFC_E_INVALID, std::string(who) + ": null handle");
  if (lfc_status st = check_device(lf, who)) return st;
  if (n < 0 || n > 65535) return fail(LFC_E_INVALID, std::string(who) + ": n must be 0..65535");
  if (out_w < 1 || out_h < 1 || out_w > 16384 || out_h > 16384)
    return fail(LFC_E_INVALID, std::string(who) + ": out_w and out_h must be 1..16384");
  if (n == 0) return LFC_OK;
  if (lfc_status st = check_buffer(d_views, (size_t)n * sizeof(lfc_view), 4, who, "d_views")) return st;
  return check_buffer(d_out, (size_t)n * 3 * out_h * out_w * 4, 4, who, "d_out");
}

}  // namespace

extern "C" lfc_status lfc_decode_blocks(const lfc_lf *lf, const int32_t *d_req, int64_t n, int32_t layout,
                                        int16_t *d_out, hipStream_t s) {
  return lfc_decode_blocks_ex(lf, d_req, n, layout, d_out, nullptr, s);
}

extern "C" lfc_status lfc_decode_blocks_ex(const lfc_lf *lf, const int32_t *d_req, int64_t n, int32_t layout,
                                           int16_t *d_out, const lfc_decode_config *cfg, hipStream_t s) {
  const char *who = "lfc_decode_blocks";
  const int64_t stage_cap = cfg ? cfg->stage_cap_words : (lf ? lf->stage_cap : 0);
  if (stage_cap < -1) return fail(LFC_E_INVALID, "lfc_decode_blocks: stage_cap_words must be >= -1");
  if (!lf) return fail(LFC_E_INVALID, "lfc_decode_blocks: null handle");
  if (lfc_status st = check_device(lf, who)) return st;
  const lfc::Geometry &g = lf->geo;
  if (n < 0) return fail(LFC_E_INVALID, "lfc_decode_blocks: n < 0");
  if (layout == LFC_LAYOUT_IMAGES) {
    if (d_req) return fail(LFC_E_INVALID, "lfc_decode_blocks: the images layout decodes every block (d_req must be NULL)");
    if (n != g.nv()) return fail(LFC_E_INVALID, "lfc_decode_blocks: images layout needs n == grid_u*grid_v");
    if (lfc_status st = check_buffer(d_out, (size_t)g.nv() * 3 * g.hp * g.wp * 2, 16, who, "d_out")) return st;
    switch (g.B) {
      case 2: return decode_images<2>(lf, d_out, s, stage_cap);
      case 4: return decode_images<4>(lf, d_out, s, stage_cap);
      default: return decode_images<8>(lf, d_out, s, stage_cap);
    }
  }
  if (layout != LFC_LAYOUT_BLOCKS) return fail(LFC_E_INVALID, "lfc_decode_blocks: unknown layout");
  if (n == 0) return LFC_OK;
  if (!d_req && n != (int64_t)g.nv() * g.nb)
    return fail(LFC_E_INVALID, "lfc_decode_blocks: with d_req NULL, n must be grid_u*grid_v*n_blocks");
  if (d_req)
    if (lfc_status st = check_buffer(d_req, (size_t)n * 8, 4, who, "d_req")) return st;
  if (lfc_status st = check_buffer(d_out, (size_t)n * 3 * g.S * 2, 16, who, "d_out")) return st;
  switch (g.B) {
    case 2: return decode_list<2>(lf, d_req, n, d_out, s);
    case 4: return decode_list<4>(lf, d_req, n, d_out, s);
    default: return decode_list<8>(lf, d_req, n, d_out, s);
  }
}

extern "C" lfc_status lfc_decode_rgb(const lfc_lf *lf, uint32_t *d_out, hipStream_t s) {
  const char *who = "lfc_decode_rgb";
  if (!lf) return fail(LFC_E_INVALID, "lfc_decode_rgb: null handle");
  if (lfc_status st = check_device(lf, who)) return st;
  if (lfc_status st = check_buffer(d_out, rgb_bytes(lf->geo), 16, who, "d_out")) return st;
  switch (lf->geo.B) {
    case 2: return decode_rgb<2>(lf, d_out, nullptr, s, who);
    case 4: return decode_rgb<4>(lf, d_out, nullptr, s, who);
    default: return decode_rgb<8>(lf, d_out, nullptr, s, who);
  }
}

extern "C" lfc_status lfc_decode_progressive(const lfc_lf *lf, const int32_t *d_req, int64_t n, int32_t level,
                                             int16_t *d_out, hipStream_t s) {
  const char *who = "lfc_decode_progressive";
  if (!lf) return fail(LFC_E_INVALID, "lfc_decode_progressive: null handle");
  if (lfc_status st = check_device(lf, who)) return st;
  const lfc::Geometry &g = lf->geo;
  if (n < 0) return fail(LFC_E_INVALID, "lfc_decode_progressive: n < 0");
  if (level < 0 || level >= g.L) return fail(LFC_E_INVALID, "lfc_decode_progressive: level must be 0..levels-1");
  if (n == 0) return LFC_OK;
  if (!d_req && n != (int64_t)g.nv() * g.nb)
    return fail(LFC_E_INVALID, "lfc_decode_progressive: with d_req NULL, n must be grid_u*grid_v*n_blocks");
  if (d_req)
    if (lfc_status st = check_buffer(d_req, (size_t)n * 8, 4, who, "d_req")) return st;
  if (lfc_status st = check_buffer(d_out, (size_t)n * 3 * g.S * 2, 16, who, "d_out")) return st;
  switch (g.B) {
    case 2: return decode_list<2>(lf, d_req, n, d_out, s, level);
    case 4: return decode_list<4>(lf, d_req, n, d_out, s, level);
    default: return decode_list<8>(lf, d_req, n, d_out, s, level);
  }
}

extern "C" lfc_status lfc_render_views(const lfc_lf *lf, const lfc_view *d_views, int32_t n, int32_t out_w,
                                       int32_t out_h, float *d_out, hipStream_t s) {
  return lfc_render_views_ex(lf, d_views, n, out_w, out_h, d_out, nullptr, s);
}

extern "C" lfc_status lfc_render_views_ex(const lfc_lf *lf, const lfc_view *d_views, int32_t n, int32_t out_w,
                                          int32_t out_h, float *d_out, const lfc_render_config *cfg, hipStream_t s) {
  const char *who = "lfc_render_views";
  if (lfc_status st = check_render(lf, d_views, n, out_w, out_h, d_out, who)) return st;
  if (n == 0) return LFC_OK;
  RenderChoice rc;
  if (lfc_status st = choose_render(lf, n, out_w, out_h, cfg, rc, who)) return st;
  return render_any(lf, d_views, n, out_w, out_h, d_out, rc, nullptr, s);
}

namespace {

// Device address of `scratch` on the current device, looked up once per
// device (the first call on a device) and kept.
lfc_status noalloc_scratch(void **out, const char *who) {
  constexpr int kDevices = 64;
  static std::atomic<void *> ptrs[kDevices];
  static std::mutex mu;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return fail(LFC_E_HIP, std::string(who) + ": no current device");
  if (dev >= kDevices) return fail(LFC_E_UNSUPPORTED, std::string(who) + ": device index above 63");
  void *p = ptrs[dev].load(std::memory_order_acquire);
  if (!p) {
    std::lock_guard<std::mutex> lock(mu);
    p = ptrs[dev].load(std::memory_order_relaxed);
    if (!p) {
      const hipError_t he = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (he != hipSuccess || !p) {
        (void)hipGetLastError();
        return fail(LFC_E_HIP, std::string(who) + ": address of the static scratch: " + hipGetErrorString(he));
      }
      ptrs[dev].store(p, std::memory_order_release);
    }
  }
  *out = p;
  return LFC_OK;
}

}  // namespace

extern "C" lfc_status lfc_render_views_noalloc(const lfc_lf *lf, const lfc_view *d_views, int32_t n, int32_t out_w,
                                               int32_t out_h, float *d_out, const lfc_render_config *cfg,
                                               hipStream_t s) {
  const char *who = "lfc_render_views_noalloc";
  if (lfc_status st = check_render(lf, d_views, n, out_w, out_h, d_out, who)) return st;
  if (n == 0) return LFC_OK;
  RenderChoice rc;
  if (lfc_status st = choose_render(lf, n, out_w, out_h, cfg, rc, who)) return st;
  const size_t need = decoded_bytes(lf->geo);
  if (rc.decoded && need > (size_t)LFC_NOALLOC_SCRATCH_BYTES) {
    if (cfg && cfg->path == LFC_RENDER_DECODED)
      return fail(LFC_E_RANGE, std::string(who) + ": the decoded views need " + std::to_string(need) +
                                   " bytes; the static scratch holds " + std::to_string(LFC_NOALLOC_SCRATCH_BYTES));
    // the automatic choice falls back to the tile path, which needs no scratch
    RenderChoice tiles = rc;
    lfc_render_config tc{LFC_RENDER_TILES, 0, 0, rc.disp};
    if (lfc_status st = choose_render(lf, n, out_w, out_h, &tc, tiles, who)) return st;
    rc = tiles;
  }
  void *ws = nullptr;
  if (rc.decoded)
    if (lfc_status st = noalloc_scratch(&ws, who)) return st;
  return render_any(lf, d_views, n, out_w, out_h, d_out, rc, ws, s);
}

// Measured tuning: every candidate launch shape timed on the caller's views.
extern "C" lfc_status lfc_render_tune(const lfc_lf *lf, const lfc_view *d_views, int32_t n, int32_t out_w,
                                      int32_t out_h, float *d_out, int32_t reps, lfc_render_tuning *res,
                                      hipStream_t s) {
  const char *who = "lfc_render_tune";
  if (!res) return fail(LFC_E_INVALID, "lfc_render_tune: null result");
  if (lfc_status st = check_render(lf, d_views, n, out_w, out_h, d_out, who)) return st;
  if (n < 1 || reps < 1 || reps > 1000) return fail(LFC_E_INVALID, "lfc_render_tune: need n >= 1 and reps 1..1000");
  std::memset(res, 0, sizeof *res);
  static const int kShapes[][2] = {{32, 8}, {32, 16}, {64, 8}, {64, 16}, {64, 32}, {128, 8}, {128, 16}, {256, 8}};
  std::vector<lfc_render_config> cands;
  cands.push_back(lfc_render_config{LFC_RENDER_DECODED, 0, 0, 0.0f});
  for (const auto &sh : kShapes) {
    RenderPlan pl;
    if (plan_render(lf->geo, out_w, out_h, pl, sh[0], sh[1], false))
      cands.push_back(lfc_render_config{LFC_RENDER_TILES, sh[0], sh[1], 0.0f});
  }
  void *ws = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  lfc_status st = LFC_OK;
  if (hipMalloc(&ws, decoded_bytes(lf->geo)) != hipSuccess) {
    ws = nullptr;
    (void)hipGetLastError();      // clear the failed allocation's error
    cands.erase(cands.begin());   // no room for the decoded views: tile shapes only
  }
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) st = fail(LFC_E_HIP, "lfc_render_tune: events");
  float best = 0.0f;
  for (size_t i = 0; st == LFC_OK && i < cands.size() && res->n_tried < LFC_TUNE_MAX; i++) {
    RenderChoice rc;
    if (choose_render(lf, n, out_w, out_h, &cands[i], rc, who) != LFC_OK) continue;
    st = render_any(lf, d_views, n, out_w, out_h, d_out, rc, ws, s);   // warm-up
    if (st == LFC_OK && hipEventRecord(e0, s) != hipSuccess) st = fail(LFC_E_HIP, "lfc_render_tune: event record");
    for (int r = 0; st == LFC_OK && r < reps; r++) st = render_any(lf, d_views, n, out_w, out_h, d_out, rc, ws, s);
    float ms = 0.0f;
    if (st == LFC_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                         hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      st = fail(LFC_E_HIP, "lfc_render_tune: timing");
    if (st != LFC_OK) break;
    const int k = res->n_tried++;
    res->cfg[k] = cands[i];
    res->ms[k] = ms / (float)reps;
    if (k == 0 || res->ms[k] < best) {
      best = res->ms[k];
      res->best = k;
    }
  }
  if (st == LFC_OK && res->n_tried == 0) st = fail(LFC_E_UNSUPPORTED, "lfc_render_tune: no launch shape fits this output");
  if (hipStreamSynchronize(s) != hipSuccess && st == LFC_OK) st = fail(LFC_E_HIP, "lfc_render_tune: synchronize");
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (ws) (void)hipFree(ws);
  return st;
}

// A render with everything fixed at creation, optionally captured in a graph.
struct lfc_render_plan {
  const lfc_lf *lf = nullptr;
  const lfc_view *views = nullptr;
  float *out = nullptr;
  int32_t n = 0, w = 0, h = 0;
  RenderChoice rc{};
  void *ws = nullptr;               // decoded views and their mask (decoded path)
  hipStream_t cap = nullptr;        // stream the graph was captured on
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" void lfc_render_plan_destroy(lfc_render_plan *p) {
  if (!p) return;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->cap) (void)hipStreamDestroy(p->cap);
  if (p->ws) (void)hipFree(p->ws);
  delete p;
}

extern "C" lfc_status lfc_render_plan_create(const lfc_lf *lf, const lfc_render_config *cfg, const lfc_view *d_views,
                                             int32_t n, int32_t out_w, int32_t out_h, float *d_out, int32_t graph,
                                             lfc_render_plan **out) {
  const char *who = "lfc_render_plan_create";
  if (!out) return fail(LFC_E_INVALID, "lfc_render_plan_create: null result");
  *out = nullptr;
  if (lfc_status st = check_render(lf, d_views, n, out_w, out_h, d_out, who)) return st;
  if (n < 1) return fail(LFC_E_INVALID, "lfc_render_plan_create: n must be 1..65535");
  lfc_render_plan *p = new (std::nothrow) lfc_render_plan;
  if (!p) return fail(LFC_E_NOMEM, "lfc_render_plan_create: out of host memory");
  p->lf = lf;
  p->views = d_views;
  p->out = d_out;
  p->n = n;
  p->w = out_w;
  p->h = out_h;
  lfc_status st = choose_render(lf, n, out_w, out_h, cfg, p->rc, who);
  if (st == LFC_OK && p->rc.decoded) {
    hipError_t he = hipMalloc(&p->ws, decoded_bytes(lf->geo));
    if (he != hipSuccess) {
      p->ws = nullptr;
      st = fail(he == hipErrorOutOfMemory ? LFC_E_NOMEM : LFC_E_HIP, "lfc_render_plan_create: decoded views");
    }
  }
  if (st == LFC_OK && graph) {
    (void)max_lds_bytes();   // device queries done before the capture
    (void)device_cus();
    if (hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking) != hipSuccess) {
      p->cap = nullptr;
      st = fail(LFC_E_HIP, "lfc_render_plan_create: capture stream");
    } else if (hipStreamBeginCapture(p->cap, hipStreamCaptureModeRelaxed) != hipSuccess) {
      st = fail(LFC_E_HIP, "lfc_render_plan_create: begin capture");
    } else {
      st = render_any(lf, d_views, n, out_w, out_h, d_out, p->rc, p->ws, p->cap);
      hipGraph_t g = nullptr;
      const hipError_t he = hipStreamEndCapture(p->cap, &g);
      p->graph = g;
      if (st == LFC_OK && (he != hipSuccess || !g)) st = fail(LFC_E_HIP, "lfc_render_plan_create: end capture");
      if (st == LFC_OK && hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess) {
        p->exec = nullptr;
        st = fail(LFC_E_HIP, "lfc_render_plan_create: graph instantiation");
      }
    }
  }
  if (st != LFC_OK) {
    lfc_render_plan_destroy(p);
    return st;
  }
  *out = p;
  return LFC_OK;
}

extern "C" lfc_status lfc_render_plan_launch(lfc_render_plan *p, hipStream_t s) {
  if (!p) return fail(LFC_E_INVALID, "lfc_render_plan_launch: null plan");
  if (lfc_status st = check_device(p->lf, "lfc_render_plan_launch")) return st;
  if (p->exec) {
    if (hipGraphLaunch(p->exec, s) != hipSuccess) return fail(LFC_E_HIP, "lfc_render_plan_launch: graph launch");
    return LFC_OK;
  }
  return render_any(p->lf, p->views, p->n, p->w, p->h, p->out, p->rc, p->ws, s);
}

extern "C" lfc_status lfc_render_plan_info(const lfc_render_plan *p, lfc_render_config *cfg, int32_t *graph) {
  if (!p || !cfg || !graph) return fail(LFC_E_INVALID, "lfc_render_plan_info: null argument");
  *cfg = p->rc.decoded ? lfc_render_config{LFC_RENDER_DECODED, 0, 0, p->rc.disp}
                       : lfc_render_config{LFC_RENDER_TILES, p->rc.pl.TX, p->rc.pl.TY, p->rc.disp};
  *graph = p->exec != nullptr;
  return LFC_OK;
}

namespace lfc {

lfc_status scratch_alloc(void **p, size_t bytes, hipStream_t s) {
  *p = nullptr;
  hipMemPool_t pl = scratch_pool();
  const hipError_t he = pl ? hipMallocFromPoolAsync(p, bytes, pl, s) : hipMallocAsync(p, bytes, s);
  if (he != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return LFC_E_NOMEM;
  }
  return LFC_OK;
}

lfc_status device_buffer(const void *p, size_t need, size_t align, const char *who, const char *what) {
  return check_buffer(p, need, align, who, what);
}

size_t render_req_bytes() { return sizeof(RenderReq); }

size_t lf_table_bytes() { return sizeof(RAArgs); }

int lf_block(const lfc_lf *lf) { return lf->geo.B; }

void lf_table_fill(const lfc_lf *lf, void *dst) {
  const RAArgs r = ra_args(lf);
  std::memcpy(dst, &r, sizeof r);
}

lfc_status decode_multi_launch(int block, const void *d_lfs, int n_lf, const int32_t *d_req, int64_t n, int16_t *out,
                               int32_t *err, hipStream_t s) {
  if (n <= 0) return LFC_OK;
  MultiArgs a{static_cast<const RAArgs *>(d_lfs), n_lf, d_req, out, err, n};
  const int rpw = 64 / (3 * block);
  const int64_t waves = (n + rpw - 1) / rpw;
  const int64_t blocks = (waves + kThreads / 64 - 1) / (kThreads / 64);
  if (blocks > 0x7FFFFFFF) return fail(LFC_E_INVALID, "lfc_batch_decode: too many requests");
  switch (block) {
    case 2: hipLaunchKernelGGL(k_decode_multi<2>, dim3((unsigned)blocks), dim3(kThreads), 0, s, a); break;
    case 4: hipLaunchKernelGGL(k_decode_multi<4>, dim3((unsigned)blocks), dim3(kThreads), 0, s, a); break;
    default: hipLaunchKernelGGL(k_decode_multi<8>, dim3((unsigned)blocks), dim3(kThreads), 0, s, a); break;
  }
  return launched("lfc_batch_decode");
}

int lf_device(const lfc_lf *lf) { return lf->device; }

lfc_status render_req_fill(const lfc_lf *lf, const lfc_view &v, int wo, int ho, float *out, void *dst, int *block,
                           int *ntiles, size_t *lds) {
  const Geometry &g = lf->geo;
  RenderPlan pl;
  if (!plan_render(g, wo, ho, pl))
    return fail(LFC_E_UNSUPPORTED, "lfc_batch_render: output too strongly minified for the tile footprint");
  RenderReq r{};
  r.a = RenderArgs{ra_args(lf), nullptr, out, wo, ho, g.U, g.V, g.W, g.H, pl.TX, pl.TY, pl.fbx, pl.fby, 0.0f};
  r.view = v;
  r.ntx = (wo + pl.TX - 1) / pl.TX;
  r.ntiles = r.ntx * ((ho + pl.TY - 1) / pl.TY);
  std::memcpy(dst, &r, sizeof r);
  *block = g.B;
  *ntiles = r.ntiles;
  *lds = pl.lds;
  return LFC_OK;
}

// ---- the colour decode-then-interpolate path of a batch -------------------

namespace {

// LDS words of the key-view rows of a colour strip, or 0 when they exceed the
// kernel's staging budget (then read from global memory)
int rgb_key_words(const lfc::Geometry &g) {
  const int64_t kw = (int64_t)3 * g.n_top * g.B * 32;
  return kw <= kRGBKeyWordsMax ? (int)kw : 0;
}

int rgb_parts(const lfc_lf *lf) {
  const lfc::Geometry &g = lf->geo;
  const int nblk = 64 / g.B, nstrips = g.nby * ((g.nbx + nblk - 1) / nblk);
  return std::max(1, std::min(lf->rgb_max_chunks, (3 * 3 * device_cus() + nstrips - 1) / nstrips));
}

}  // namespace

bool lf_rgb_batchable(const lfc_lf *lf, double out_pixels) {
  const Geometry &g = lf->geo;
  const size_t lds = 4 * ((size_t)kRGBHeadWords + (size_t)lf_tile_words(lf->tile_cap_rgb, g.B * g.B) +
                          (size_t)rgb_key_words(g));
  return (uint64_t)g.nv() * g.hp * g.wp * 4 < ((uint64_t)1 << 32) && g.nv() <= 32 * kRGBNeedWords &&
         lds <= (size_t)max_lds_bytes() && 20.0 * out_pixels >= (double)g.nv() * g.hp * g.wp;
}

size_t lf_rgb_bytes(const lfc_lf *lf) { return rgb_bytes(lf->geo); }

int lf_rgb_items(const lfc_lf *lf) {
  const Geometry &g = lf->geo;
  const int nblk = 64 / g.B;
  return g.nby * ((g.nbx + nblk - 1) / nblk) * rgb_parts(lf);
}

int lf_views(const lfc_lf *lf) { return lf->geo.nv(); }

size_t rgb_args_bytes() { return sizeof(RGBArgs); }

void rgb_args_fill(const lfc_lf *lf, bool keys, uint32_t *d_rgb, const uint32_t *d_mask, void *dst) {
  const Geometry &g = lf->geo;
  const int nblk = 64 / g.B;
  RGBArgs a{lf->d_rkv, lf->d_off, lf->d_srv, lf->d_sched_rgb, lf->d_strip_off_rgb, lf->d_order_rgb, lf->d_batch,
            d_mask, d_rgb, g.nbx, (g.nbx + nblk - 1) / nblk, g.L, g.q, g.wp, g.hp, g.nb, lf->n_batch, g.nv(),
            g.n_top, keys ? rgb_key_words(g) : 0, lf->tile_cap_rgb, rgb_parts(lf)};
  std::memcpy(dst, &a, sizeof a);
}

size_t rgb_lds_bytes(const lfc_lf *lf, bool keys) {
  const Geometry &g = lf->geo;
  return 4 * ((size_t)kRGBHeadWords + (size_t)lf_tile_words(lf->tile_cap_rgb, g.B * g.B) +
              (size_t)(keys ? rgb_key_words(g) : 0));
}

bool rgb_keys_fit(const lfc_lf *lf) { return rgb_key_words(lf->geo) > 0; }

void need_mask_host(const lfc_lf *lf, const lfc_view &v, uint32_t *mask) {
  const Geometry &g = lf->geo;
  // the grid cell the renderers read (cell() on the device, the same float
  // clamp and floor)
  auto cell_host = [](float x, int n, int &i0, int &i1) {
    x = std::fmin(std::fmax(x, 0.0f), (float)(n - 1));
    if (n == 1) {
      i0 = i1 = 0;
      return;
    }
    int i = (int)std::floor(x);
    i = std::min(std::max(i, 0), n - 2);
    i0 = i;
    i1 = i + 1;
  };
  int iu0, iu1, jv0, jv1;
  cell_host(v.u, g.U, iu0, iu1);
  cell_host(v.v, g.V, jv0, jv1);
  for (int vi : {jv0 * g.U + iu0, jv0 * g.U + iu1, jv1 * g.U + iu0, jv1 * g.U + iu1}) mask[vi >> 5] |= 1u << (vi & 31);
}

size_t interp_req_bytes() { return sizeof(InterpReq); }

void interp_req_fill(const lfc_lf *lf, const uint32_t *d_rgb, const lfc_view &v, int wo, int ho, float *out,
                     void *dst) {
  const Geometry &g = lf->geo;
  InterpReq r{};
  r.a = InterpRGBArgs{d_rgb, (uint32_t)rgb_bytes(g), nullptr, out, wo, ho, g.U, g.V, g.W, g.H, g.wp, g.hp, 0.0f,
                      (float)g.W / (float)wo, (float)g.H / (float)ho};
  r.view = v;
  std::memcpy(dst, &r, sizeof r);
}

lfc_status rgb_multi_launch(int block, bool keys, const void *d_args, const int32_t *d_first, int n_lf, int n_items,
                            size_t lds, uint32_t *d_ctr, hipStream_t s) {
  if (n_items <= 0) return LFC_OK;
  RGBMultiArgs m{static_cast<const RGBArgs *>(d_args), d_first, n_lf, n_items, d_ctr};
  // resident workgroups: as many as the compute units hold at this LDS size
  auto launch = [&](auto kern) -> lfc_status {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kLFThreads, lds) != hipSuccess || per_cu < 1) {
      (void)hipGetLastError();
      per_cu = 1;
    }
    const int grid = std::max(1, std::min(n_items, per_cu * device_cus()));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kLFThreads), lds, s, m);
    return launched("lfc_batch_render");
  };
  switch (block * 2 + (keys ? 1 : 0)) {
    case 5: return launch(k_decode_rgb_multi<2, true>);
    case 4: return launch(k_decode_rgb_multi<2, false>);
    case 9: return launch(k_decode_rgb_multi<4, true>);
    case 8: return launch(k_decode_rgb_multi<4, false>);
    case 17: return launch(k_decode_rgb_multi<8, true>);
    default: return launch(k_decode_rgb_multi<8, false>);
  }
}

lfc_status interp_multi_launch(const void *d_reqs, int n, int max_wo, int max_ho, hipStream_t s) {
  if (n <= 0) return LFC_OK;
  if (n > 65535) return fail(LFC_E_INVALID, "lfc_batch_render: at most 65535 interpolated requests per batch");
  const dim3 grid((unsigned)((max_wo + kThreads - 1) / kThreads), (unsigned)n, (unsigned)max_ho);
  hipLaunchKernelGGL(k_interp_multi, grid, dim3(kThreads), 0, s, static_cast<const InterpReq *>(d_reqs));
  return launched("lfc_batch_render");
}

lfc_status render_multi_launch(int block, const void *d_reqs, int n, int max_tiles, size_t lds, hipStream_t s) {
  if (n <= 0) return LFC_OK;
  if (n > 65535) return fail(LFC_E_INVALID, "lfc_batch_render: at most 65535 requests of one block size per batch");
  const RenderReq *r = static_cast<const RenderReq *>(d_reqs);
  dim3 grid((unsigned)max_tiles, (unsigned)n);
  switch (block) {
    case 2: hipLaunchKernelGGL(k_render_multi<2>, grid, dim3(kRenderThreads), lds, s, r); break;
    case 4: hipLaunchKernelGGL(k_render_multi<4>, grid, dim3(kRenderThreads), lds, s, r); break;
    default: hipLaunchKernelGGL(k_render_multi<8>, grid, dim3(kRenderThreads), lds, s, r); break;
  }
  return launched("lfc_batch_render");
}

}  // namespace lfc

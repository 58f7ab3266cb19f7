// HIP kernels for gfx950 (CDNA4, wave64) and the exported launch calls
// lfc_decode_blocks and lfc_render_views.
//
// Decoding a block (Alg. 2, Sec. 3.5) is: read the top-level key-view block,
// then for every level below, locate the node's residual block inside the
// group of its spatial location (one level of indirection through the
// block offsets, Sec. 3.4), unpack its BISE values (Sec. 3.3), undo the
// zigzag and the quantiser step, and add it.  All integer work; no MFMA.
//
// Work mapping: one lane owns one row of B samples of one block of one
// channel, so a wave covers a 64-pixel-wide strip of B rows and its stores
// are full 128-byte row segments.  Samples travel as packed int16 pairs:
// the residual tail (zigzag undo, step 2^q, adding the parent) runs on both
// halves of a register at once, and the sums wrap modulo 2^16 exactly as the
// final int16 store of a 32-bit sum would.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <string>
#include <type_traits>

#include "internal.h"

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
__device__ __forceinline__ uint16_t lut_entry(int t) {
  uint32_t v = 0;
  if (t < 256) {
    if (t < 243)
      for (int r = 0, x = t; r < 5; r++, x /= 3) v |= (uint32_t)(x % 3) << (2 * r);
  } else {
    const int q = t - 256;
    if (q < 125)
      for (int r = 0, x = q; r < 3; r++, x /= 5) v |= (uint32_t)(x % 5) << (3 * r);
  }
  return (uint16_t)v;
}

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

// two zigzagged values (0,1,2,3,.. -> 0,-1,1,-2,..) back to signed, times 2^q
__device__ __forceinline__ uint32_t unzigzag_pk(uint32_t pr, int q) {
  const u16x2 x = as_u16x2(pr);
  const u16x2 one = {1, 1};
  const u16x2 zero = {0, 0};
  u16x2 r = (x >> one) ^ (zero - (x & one));
  const u16x2 sh = {(unsigned short)q, (unsigned short)q};
  return as_u32(r << sh);
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

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Inclusive prefix sum over the 64 lanes with DPP row shifts and row
// broadcasts (no LDS traffic): shifts by 1, 2, 4, 8 scan each row of 16
// lanes, then lane 15 of each row is added to the next row and lane 31 to the
// upper half.  Lanes without a source add 0.
__device__ __forceinline__ uint32_t wave_scan_dpp(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);  // row_shr:1
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);  // row_shr:2
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);  // row_shr:4
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);  // row_shr:8
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);  // row_bcast:15
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return v;
}

// ---------------------------------------------------------------------------
// whole light field, images layout
// ---------------------------------------------------------------------------

constexpr int kLFThreads = 512;
constexpr int kLFWaves = kLFThreads / 64;
constexpr int kLFHeadWords = 400;     // LDS words before the descriptors (LUT, group extents)
constexpr int kStagePad = 8;          // zero words after the staged groups

struct LFArgs {
  const int16_t *rkv;
  const uint32_t *off;
  const uint32_t *srv;
  const int32_t *batch;  // [nbatch][kBatchWords] runs of sibling leaves (see internal.h)
  int16_t *out;          // [nv][3][hp][wp]
  int nbx, n_srv, nbw, nv, L, q, wp, hp, nb, nbatch;
  int stage_cap;         // LDS words available for the strip's groups
};

// Where every node's residual block starts in group gw (or that it is absent):
// bitmap rank by ballot, 5-bit code, wave prefix sum of the block sizes.
template <int S>
__device__ __forceinline__ void scan_group(const uint32_t *gw, uint32_t len, uint32_t *dj, int n_srv, int nbw,
                                           int lane) {
  uint32_t cnt = 0;
  for (int w = lane; w < nbw; w += 64) cnt += __popc(gw[w]);
  cnt = wave_sum(cnt);
  const uint32_t code_bit0 = 32u * nbw;
  uint32_t rank_base = 0, bit_base = 32u * (nbw + (5u * cnt + 31u) / 32u);
  for (int s0 = 0; s0 < n_srv; s0 += 64) {
    const int s = s0 + lane;
    const bool pres = s < n_srv && ((gw[s >> 5] >> (s & 31)) & 1u);
    const uint64_t bal = __ballot(pres);
    const uint32_t rank = rank_base + __popcll(bal & ((1ull << lane) - 1ull));
    uint32_t code = 0, size = 0;
    if (pres) {
      code = (uint32_t)window64(gw, code_bit0 + 5u * rank) & 31u;
      size = block_bits<S>(code);
    }
    const uint32_t incl = wave_scan_dpp(size);
    // a block starts inside its group; the clamp keeps every later read there
    const uint32_t at = min(bit_base + incl - size, 32u * len);
    if (s < n_srv) dj[s] = pres ? ((at << 5) | code) : kAbsent;
    rank_base += __popcll(bal);
    bit_base += (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
  }
}

// LDS written by some lanes of a wave and read by others of the same wave:
// order the accesses (LDS instructions of one wave complete in order).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Per-wave LDS scratch of phase B: the list of stored (sibling, lane) rows
// and their decoded residuals.
template <int B>
struct PhaseBScratch {
  static constexpr int kListWords = lfc::kBatch * 64 / 2;      // u16 items
  static constexpr int kResWords = lfc::kBatch * 64 * (B / 2);
  static constexpr int kWords = kListWords + kResWords;
};

// Phase B of the whole-field kernel for one wave: a run of sibling batches in
// serial order (one 64-byte scalar record each).  The reconstruction of every
// ancestor level of the current batch is kept in registers (T[t], t =
// top..4), so a parent's residual is decoded once per subtree.  For the
// leaves, the rows whose block is stored are first listed in LDS and decoded
// densely (about a third of them at 40 dB), then every lane adds its row's
// residual, if any, to the parent and stores.
template <int B>
__device__ __forceinline__ void lf_leaves(const LFArgs &a, const uint32_t *base, const uint32_t *goff,
                                          const uint32_t *desc, const uint32_t *plans, uint32_t *scratch,
                                          const uint16_t *lut, int wave, int lane) {
  constexpr int S = B * B, NBLK = 64 / B, H = B / 2;
  const int j = lane % NBLK, y = lane / NBLK;
  const int bx = blockIdx.x * NBLK + j, by = blockIdx.y, c = blockIdx.z;
  const bool active = bx < a.nbx;
  const int b = by * a.nbx + (active ? bx : 0);
  const int top = kMaxLevels - a.L;
  const size_t row = (size_t)(by * B + y) * a.wp + bx * B;
  const size_t vstride = (size_t)3 * a.hp * a.wp, cplane = (size_t)c * a.hp * a.wp;
  const uint32_t *dj = desc + j * a.n_srv;
  const uint32_t *gw = base + goff[j];
  const uint32_t plan_t = plans[2 * y], plan_q = plans[2 * y + 1];
  uint16_t *list = reinterpret_cast<uint16_t *>(scratch + wave * PhaseBScratch<B>::kWords);
  uint32_t *res = scratch + wave * PhaseBScratch<B>::kWords + PhaseBScratch<B>::kListWords;
  const uint64_t lanes_below = (1ull << lane) - 1ull;
  uint32_t T[kMaxLevels - 1][H];
  int cache[kMaxLevels - 1];
#pragma unroll
  for (int t = 0; t < kMaxLevels - 1; t++) cache[t] = -1;
  const int per = (a.nbatch + kLFWaves - 1) / kLFWaves;
  const int q0 = wave * per, q1 = min(a.nbatch, q0 + per);
  for (int qb = q0; qb < q1; qb++) {
    const int32_t *rec = a.batch + (size_t)qb * lfc::kBatchWords;
    bool changed = false;
#pragma unroll
    for (int t = 0; t < kMaxLevels - 1; t++) {
      if (t < top) continue;
      if (t == top) {
        const int root = rec[5];
        changed = root != cache[t];
        if (changed) {
          cache[t] = root;
          if (active) load_row<B>(a.rkv + ((size_t)(root * a.nb + b) * 3 + c) * S + y * B, T[t]);
          else
#pragma unroll
            for (int i = 0; i < H; i++) T[t][i] = 0;
        }
      } else {
        const int s = rec[6 + t - top - 1];
        changed = changed || s != cache[t];
        if (changed) {
          cache[t] = s;
          const uint32_t e = dj[s];
          uint32_t d[H];
          if (e != kAbsent) decode_row<B>(gw, e, plan_t, plan_q, y, a.q, lut, d);
          else
#pragma unroll
            for (int i = 0; i < H; i++) d[i] = 0;
#pragma unroll
          for (int i = 0; i < H; i++) T[t][i] = add_pk(T[t > 0 ? t - 1 : 0][i], d[i]);
        }
      }
    }
    const int nsib = rec[0], s0 = rec[10];
    bool stored[lfc::kBatch];
    uint32_t cnt = 0;
#pragma unroll
    for (int i = 0; i < lfc::kBatch; i++) {
      stored[i] = i < nsib && dj[s0 + i] != kAbsent;
      const uint64_t bal = __ballot(stored[i]);
      if (stored[i]) list[cnt + __popcll(bal & lanes_below)] = (uint16_t)(i * 64 + lane);
      cnt += __popcll(bal);
    }
    wave_lds_sync();
    for (uint32_t p0 = 0; p0 < cnt; p0 += 64) {
      if (p0 + lane < cnt) {
        const uint32_t item = list[p0 + lane];
        const int i2 = item >> 6, l2 = item & 63, j2 = l2 % NBLK, y2 = l2 / NBLK;
        uint32_t d[H];
        decode_row<B>(base + goff[j2], desc[j2 * a.n_srv + s0 + i2], plans[2 * y2], plans[2 * y2 + 1], y2, a.q,
                      lut, d);
#pragma unroll
        for (int h = 0; h < H; h++) res[item * H + h] = d[h];
      }
    }
    wave_lds_sync();
#pragma unroll
    for (int i = 0; i < lfc::kBatch; i++) {
      if (i < nsib) {
        uint32_t x[H];
#pragma unroll
        for (int h = 0; h < H; h++) x[h] = T[kMaxLevels - 2][h];
        if (stored[i])
#pragma unroll
          for (int h = 0; h < H; h++) x[h] = add_pk(x[h], res[(i * 64 + lane) * H + h]);
        if (active) store_row<B>(a.out + (size_t)rec[1 + i] * vstride + cplane + row, x);
      }
    }
    wave_lds_sync();
  }
}

// One workgroup = one channel c, one row of blocks by, one strip of 64/B
// consecutive blocks (64 pixels).  Phase A copies the strip's groups into
// LDS when they fit (else phase B reads them from global memory) and writes,
// for every tree node and block, where its residual block starts.  Phase B
// walks the leaves (lf_leaves), 8 waves splitting them.
template <int B>
__global__ __launch_bounds__(kLFThreads) void k_decode_lf(LFArgs a) {
  constexpr int S = B * B, NBLK = 64 / B;
  extern __shared__ uint32_t smem[];
  uint16_t *lut = reinterpret_cast<uint16_t *>(smem);  // 384 x u16 = 192 words
  uint32_t *s_o0 = smem + 192;                         // group start word in the SRV section
  uint32_t *s_len = smem + 256;                        // group length in words
  uint32_t *s_so = smem + 320;                         // group start in the staging area, and the total
  uint32_t *plans = smem + 384;                        // [B][2] digit plans per row (trit, quint)
  uint32_t *desc = smem + kLFHeadWords;                // [NBLK][n_srv]
  uint32_t *scratch = desc + NBLK * a.n_srv;           // [kLFWaves][PhaseBScratch<B>::kWords]
  uint32_t *stage = scratch + kLFWaves * PhaseBScratch<B>::kWords;  // [stage_cap + kStagePad]
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  for (int t = tid; t < kLutEntries; t += kLFThreads) lut[t] = lut_entry(t);
  if (tid < 2 * B) plans[tid] = digit_plan<B>(tid >> 1, (tid & 1) == 0);
  if (tid < NBLK) {
    const int bx = blockIdx.x * NBLK + tid;
    uint32_t o0 = 0, o1 = 0;
    if (bx < a.nbx) {
      const int g = 3 * (blockIdx.y * a.nbx + bx) + blockIdx.z;
      o0 = a.off[g];
      o1 = a.off[g + 1];
    }
    s_o0[tid] = o0;
    s_len[tid] = o1 - o0;
  }
  __syncthreads();
  if (tid == 0) {
    uint32_t acc = 0;
    for (int j = 0; j < NBLK; j++) {
      s_so[j] = acc;
      acc += s_len[j];
    }
    s_so[NBLK] = acc;
  }
  __syncthreads();
  const uint32_t total = s_so[NBLK];
  const bool staged = total <= (uint32_t)a.stage_cap;
  if (staged) {
    for (int j = wave; j < NBLK; j += kLFWaves) {
      const uint32_t *src = a.srv + s_o0[j];
      uint32_t *dst = stage + s_so[j];
      const uint32_t n = s_len[j];
      for (uint32_t i = lane; i < n; i += 256) {
        // four loads in flight per lane before the stores
        uint32_t v[4];
#pragma unroll
        for (int u = 0; u < 4; u++) v[u] = i + 64 * u < n ? src[i + 64 * u] : 0u;
#pragma unroll
        for (int u = 0; u < 4; u++)
          if (i + 64 * u < n) dst[i + 64 * u] = v[u];
      }
    }
    if (tid < kStagePad) stage[total + tid] = 0;
  }
  __syncthreads();
  for (int j = wave; j < NBLK; j += kLFWaves) {
    uint32_t *dj = desc + j * a.n_srv;
    if (s_len[j] == 0) {
      for (int s = lane; s < a.n_srv; s += 64) dj[s] = kAbsent;
      continue;
    }
    if (staged) scan_group<S>(stage + s_so[j], s_len[j], dj, a.n_srv, a.nbw, lane);
    else scan_group<S>(a.srv + s_o0[j], s_len[j], dj, a.n_srv, a.nbw, lane);
  }
  __syncthreads();
  const int j = lane % NBLK;
  if (a.L == 1) {
    // no residual levels: every view is a stored key view
    const int y = lane / NBLK, bx = blockIdx.x * NBLK + j;
    if (bx >= a.nbx) return;
    const int b = blockIdx.y * a.nbx + bx;
    const int per = (a.nbatch + kLFWaves - 1) / kLFWaves;
    for (int qb = wave * per; qb < min(a.nbatch, wave * per + per); qb++) {
      const int32_t *rec = a.batch + (size_t)qb * lfc::kBatchWords;
      uint32_t x[B / 2];
      load_row<B>(a.rkv + ((size_t)(rec[5] * a.nb + b) * 3 + blockIdx.z) * S + y * B, x);
      store_row<B>(a.out + ((size_t)(rec[1] * 3 + blockIdx.z) * a.hp + blockIdx.y * B + y) * a.wp + bx * B, x);
    }
    return;
  }
  if (staged) lf_leaves<B>(a, stage, s_so, desc, plans, scratch, lut, wave, lane);
  else lf_leaves<B>(a, a.srv, s_o0, desc, plans, scratch, lut, wave, lane);
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
};

// Row y of block b, channel c, of view vi (Alg. 2): key-view row plus the
// residual rows of the view's ancestors, as B/2 packed int16 pairs.
template <int B>
__device__ __forceinline__ void gather_row(const RAArgs &a, int vi, int b, int c, int y, uint32_t plan_t,
                                           uint32_t plan_q, const uint16_t *lut, uint32_t x[B / 2]) {
  constexpr int S = B * B;
  const int root = a.root[vi];
  load_row<B>(a.rkv + ((size_t)(root * a.nb + b) * 3 + c) * S + y * B, x);
  const int g = 3 * b + c;
  const uint32_t o0 = a.off[g], o1 = a.off[g + 1];
  if (o0 == o1) return;
  const uint32_t *gw = a.srv + o0;
  const int depth = a.L - 1;
  for (int l = depth - 1; l >= 0; --l) {
    const int s = a.path[vi * depth + l];
    const uint32_t bm = gw[s >> 5];
    const uint32_t bit = (uint32_t)s & 31u;
    if ((bm >> bit) & 1u) {
      const uint32_t idx = a.dbase[(size_t)g * a.nbw + (s >> 5)] + __popc(bm & ((1u << bit) - 1u));
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
    gather_row<B>(a.ra, vi, b, c, y, digit_plan<B>(y, true), digit_plan<B>(y, false), lut, x);
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

template <int B>
__global__ __launch_bounds__(kThreads) void k_render(RenderArgs a) {
  extern __shared__ uint32_t smem[];
  uint16_t *lut = reinterpret_cast<uint16_t *>(smem);
  uint32_t *rgb = smem + kLutEntries / 2;      // [4][fby_max*B][fbx_max*B], packed R | G<<8 | B<<16
  const int tid = threadIdx.x;
  for (int t = tid; t < kLutEntries; t += kThreads) lut[t] = lut_entry(t);
  const int n = blockIdx.z;
  const lfc_view vw = a.views[n];
  int iu0, iu1, jv0, jv1;
  float fu, fv;
  cell(vw.u, a.U, iu0, iu1, fu);
  cell(vw.v, a.V, jv0, jv1, fv);
  const float sxs = (float)a.W / (float)a.wo, tys = (float)a.H / (float)a.ho;
  const int tx0 = blockIdx.x * a.TX, ty0 = blockIdx.y * a.TY;
  const int tx1 = min(tx0 + a.TX, a.wo) - 1, ty1 = min(ty0 + a.TY, a.ho) - 1;
  // source footprint of the tile, one pixel wider on each side than needed
  const float sa = fminf(fmaxf(vw.s + ((float)tx0 + 0.5f) * sxs - 0.5f, 0.0f), (float)(a.W - 1));
  const float sb = fminf(fmaxf(vw.s + ((float)tx1 + 0.5f) * sxs - 0.5f, 0.0f), (float)(a.W - 1));
  const float ta = fminf(fmaxf(vw.t + ((float)ty0 + 0.5f) * tys - 0.5f, 0.0f), (float)(a.H - 1));
  const float tb = fminf(fmaxf(vw.t + ((float)ty1 + 0.5f) * tys - 0.5f, 0.0f), (float)(a.H - 1));
  const int xlo = max((int)floorf(sa) - 1, 0), xhi = min((int)floorf(sb) + 2, a.W - 1);
  const int ylo = max((int)floorf(ta) - 1, 0), yhi = min((int)floorf(tb) + 2, a.H - 1);
  const int fbx0 = xlo / B, fby0 = ylo / B;
  const int FBX = min(xhi / B - fbx0 + 1, a.fbx_max), FBY = min(yhi / B - fby0 + 1, a.fby_max);
  const int FW = a.fbx_max * B, FH = a.fby_max * B;
  int vis[4];
  vis[0] = jv0 * a.U + iu0;
  vis[1] = jv0 * a.U + iu1;
  vis[2] = jv1 * a.U + iu0;
  vis[3] = jv1 * a.U + iu1;
  __syncthreads();

  // decode the footprint: item = (view k, block row fy, block column fx, row y)
  const int per_view = FBY * FBX * B;
  for (int it = tid; it < 4 * per_view; it += kThreads) {
    const int k = it / per_view, rem = it - k * per_view;
    const int fy = rem / (FBX * B), rem2 = rem - fy * FBX * B;
    const int fx = rem2 / B, y = rem2 - fx * B;
    const int b = (fby0 + fy) * a.ra.nbx + fbx0 + fx;
    const uint32_t plan_t = digit_plan<B>(y, true), plan_q = digit_plan<B>(y, false);
    uint32_t Y[B / 2], Co[B / 2], Cg[B / 2];
    gather_row<B>(a.ra, vis[k], b, 0, y, plan_t, plan_q, lut, Y);
    gather_row<B>(a.ra, vis[k], b, 1, y, plan_t, plan_q, lut, Co);
    gather_row<B>(a.ra, vis[k], b, 2, y, plan_t, plan_q, lut, Cg);
    uint32_t *dst = rgb + (k * FH + fy * B + y) * FW + fx * B;
#pragma unroll
    for (int i = 0; i < B; i++) {
      const int32_t yv = (i & 1) ? hi16(Y[i / 2]) : lo16(Y[i / 2]);
      const int32_t co = (i & 1) ? hi16(Co[i / 2]) : lo16(Co[i / 2]);
      const int32_t cg = (i & 1) ? hi16(Cg[i / 2]) : lo16(Cg[i / 2]);
      // inverse YCoCg-R (Sec. 4), clamped to 8 bits
      const int32_t t = yv - (cg >> 1);
      const int32_t G = cg + t;
      const int32_t Bc = t - (co >> 1);
      const int32_t R = Bc + co;
      dst[i] = (uint32_t)min(max(R, 0), 255) | ((uint32_t)min(max(G, 0), 255) << 8) |
               ((uint32_t)min(max(Bc, 0), 255) << 16);
    }
  }
  __syncthreads();

  // quadrilinear interpolation of every output pixel of the tile
  const size_t plane = (size_t)a.ho * a.wo;
  float *outn = a.out + (size_t)n * 3 * plane;
  for (int p = tid; p < a.TX * a.TY; p += kThreads) {
    const int X = tx0 + p % a.TX, Yp = ty0 + p / a.TX;
    if (X >= a.wo || Yp >= a.ho) continue;
    int x0, x1, y0, y1;
    float fs, ft;
    cell(vw.s + ((float)X + 0.5f) * sxs - 0.5f, a.W, x0, x1, fs);
    cell(vw.t + ((float)Yp + 0.5f) * tys - 0.5f, a.H, y0, y1, ft);
    const int lx0 = min(max(x0 - fbx0 * B, 0), FW - 1), lx1 = min(max(x1 - fbx0 * B, 0), FW - 1);
    const int ly0 = min(max(y0 - fby0 * B, 0), FH - 1), ly1 = min(max(y1 - fby0 * B, 0), FH - 1);
    uint32_t P[4][4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const uint32_t *img = rgb + k * FH * FW;
      P[k][0] = img[ly0 * FW + lx0];
      P[k][1] = img[ly0 * FW + lx1];
      P[k][2] = img[ly1 * FW + lx0];
      P[k][3] = img[ly1 * FW + lx1];
    }
#pragma unroll
    for (int ch = 0; ch < 3; ch++) {
      float lt[4];
#pragma unroll
      for (int k = 0; k < 4; k++) {
        const float p00 = (float)((P[k][0] >> (8 * ch)) & 255u), p01 = (float)((P[k][1] >> (8 * ch)) & 255u);
        const float p10 = (float)((P[k][2] >> (8 * ch)) & 255u), p11 = (float)((P[k][3] >> (8 * ch)) & 255u);
        lt[k] = lerpf(lerpf(p00, p01, fs), lerpf(p10, p11, fs), ft);
      }
      // k = 0: (u0, v0), 1: (u1, v0), 2: (u0, v1), 3: (u1, v1)
      const float lv0 = lerpf(lt[0], lt[2], fv), lv1 = lerpf(lt[1], lt[3], fv);
      outn[ch * plane + (size_t)Yp * a.wo + X] = lerpf(lv0, lv1, fu) / 255.0f;
    }
  }
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
                g.nb, g.nbx, g.nv(), g.nbw, g.L, g.q};
}

lfc_status launched(const char *who) {
  const hipError_t he = hipGetLastError();
  if (he != hipSuccess) return fail(LFC_E_HIP, std::string(who) + ": launch failed: " + hipGetErrorString(he));
  return LFC_OK;
}

int max_lds_bytes() {
  static int cached = 0;
  if (!cached) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
      v = 64 * 1024;
    cached = v < 64 * 1024 ? v : 64 * 1024;
  }
  return cached;
}

template <int B>
lfc_status decode_images(const lfc_lf *lf, int16_t *out, hipStream_t s) {
  const lfc::Geometry &g = lf->geo;
  constexpr int NBLK = 64 / B;
  const int64_t fixed = kLFHeadWords + (int64_t)NBLK * g.n_srv + kLFWaves * PhaseBScratch<B>::kWords + kStagePad;
  const int64_t avail = max_lds_bytes() / 4 - fixed;
  if (avail < 0)
    return fail(LFC_E_UNSUPPORTED, "lfc_decode_blocks: tree too large for the whole-field kernel; use BLOCKS layout");
  int64_t cap = std::min<int64_t>(avail, lf->max_strip_words);
  if (const char *e = getenv("LFC_STAGE_CAP_WORDS")) cap = std::min<int64_t>(cap, std::max(0, atoi(e)));
  const size_t lds = 4 * (size_t)(fixed + cap);
  LFArgs a{lf->d_rkv, lf->d_off, lf->d_srv, lf->d_batch, out, g.nbx, g.n_srv, g.nbw, g.nv(), g.L, g.q, g.wp, g.hp,
           g.nb, lf->n_batch, (int)cap};
  dim3 grid((g.nbx + NBLK - 1) / NBLK, g.nby, 3);
  hipLaunchKernelGGL(k_decode_lf<B>, grid, dim3(kLFThreads), lds, s, a);
  return launched("lfc_decode_blocks");
}

template <int B>
lfc_status decode_list(const lfc_lf *lf, const int32_t *req, int64_t n, int16_t *out, hipStream_t s) {
  constexpr int RPW = 64 / (3 * B);
  BlocksArgs a{ra_args(lf), req, out, lf->d_err, n};
  const int64_t waves = (n + RPW - 1) / RPW;
  const int64_t blocks = (waves + kThreads / 64 - 1) / (kThreads / 64);
  if (blocks > 0x7FFFFFFF) return fail(LFC_E_INVALID, "lfc_decode_blocks: too many requests");
  hipLaunchKernelGGL(k_decode_blocks<B>, dim3((unsigned)blocks), dim3(kThreads), 0, s, a);
  return launched("lfc_decode_blocks");
}

// Tile of output pixels per workgroup, and the largest footprint (in blocks)
// any tile can need; shrinks the tile until the footprint fits 64 KB of LDS.
struct RenderPlan {
  int TX, TY, fbx, fby;
  size_t lds;
};

bool plan_render(const lfc::Geometry &g, int wo, int ho, RenderPlan &pl) {
  const double sxs = (double)g.W / wo, tys = (double)g.H / ho;
  int TX = 64, TY = 16;
  for (;;) {
    // footprint span: (T-1)*scale pixels plus the 1-pixel widening on each
    // side, the interpolation neighbour and float slack, then block alignment
    const int fbx = ((int)std::ceil((TX - 1) * sxs) + 5 + g.B - 1) / g.B + 2;
    const int fby = ((int)std::ceil((TY - 1) * tys) + 5 + g.B - 1) / g.B + 2;
    const size_t lds = 4 * ((size_t)kLutEntries / 2 + (size_t)4 * fbx * g.B * fby * g.B);
    if (lds <= 64 * 1024) {
      pl = RenderPlan{TX, TY, fbx, fby, lds};
      return true;
    }
    if (TY > 2) TY /= 2;
    else if (TX > 8) TX /= 2;
    else return false;
  }
}

template <int B>
lfc_status render(const lfc_lf *lf, const lfc_view *views, int32_t n, int32_t wo, int32_t ho, float *out,
                  hipStream_t s) {
  const lfc::Geometry &g = lf->geo;
  RenderPlan pl;
  if (!plan_render(g, wo, ho, pl))
    return fail(LFC_E_UNSUPPORTED, "lfc_render_views: output too strongly minified for the tile footprint");
  RenderArgs a{ra_args(lf), views, out, wo, ho, g.U, g.V, g.W, g.H, pl.TX, pl.TY, pl.fbx, pl.fby};
  dim3 grid((wo + pl.TX - 1) / pl.TX, (ho + pl.TY - 1) / pl.TY, n);
  hipLaunchKernelGGL(k_render<B>, grid, dim3(kThreads), pl.lds, s, a);
  return launched("lfc_render_views");
}

}  // namespace

extern "C" lfc_status lfc_decode_blocks(const lfc_lf *lf, const int32_t *d_req, int64_t n, int32_t layout,
                                        int16_t *d_out, hipStream_t s) {
  const char *who = "lfc_decode_blocks";
  if (!lf) return fail(LFC_E_INVALID, "lfc_decode_blocks: null handle");
  if (lfc_status st = check_device(lf, who)) return st;
  const lfc::Geometry &g = lf->geo;
  if (n < 0) return fail(LFC_E_INVALID, "lfc_decode_blocks: n < 0");
  if (layout == LFC_LAYOUT_IMAGES) {
    if (d_req) return fail(LFC_E_INVALID, "lfc_decode_blocks: the images layout decodes every block (d_req must be NULL)");
    if (n != g.nv()) return fail(LFC_E_INVALID, "lfc_decode_blocks: images layout needs n == grid_u*grid_v");
    if (lfc_status st = check_buffer(d_out, (size_t)g.nv() * 3 * g.hp * g.wp * 2, 16, who, "d_out")) return st;
    switch (g.B) {
      case 2: return decode_images<2>(lf, d_out, s);
      case 4: return decode_images<4>(lf, d_out, s);
      default: return decode_images<8>(lf, d_out, s);
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

extern "C" lfc_status lfc_render_views(const lfc_lf *lf, const lfc_view *d_views, int32_t n, int32_t out_w,
                                       int32_t out_h, float *d_out, hipStream_t s) {
  const char *who = "lfc_render_views";
  if (!lf) return fail(LFC_E_INVALID, "lfc_render_views: null handle");
  if (lfc_status st = check_device(lf, who)) return st;
  if (n < 0 || n > 65535) return fail(LFC_E_INVALID, "lfc_render_views: n must be 0..65535");
  if (out_w < 1 || out_h < 1 || out_w > 16384 || out_h > 16384)
    return fail(LFC_E_INVALID, "lfc_render_views: out_w and out_h must be 1..16384");
  if (n == 0) return LFC_OK;
  if (lfc_status st = check_buffer(d_views, (size_t)n * sizeof(lfc_view), 4, who, "d_views")) return st;
  if (lfc_status st = check_buffer(d_out, (size_t)n * 3 * out_h * out_w * 4, 4, who, "d_out")) return st;
  switch (lf->geo.B) {
    case 2: return render<2>(lf, d_views, n, out_w, out_h, d_out, s);
    case 4: return render<4>(lf, d_views, n, out_w, out_h, d_out, s);
    default: return render<8>(lf, d_views, n, out_w, out_h, d_out, s);
  }
}

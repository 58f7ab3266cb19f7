// CompressLFI (Alg. 1) on the GPU: the same stream, byte for byte, as the
// host encoder with the paper's global thresholds (lfc_encode_ex).
//
// Level 0 (YCoCg-R of the padded views, Sec. 4), the key-view filter of
// each level (eqs. 1-2), and, level by level from the top, the closed-loop
// residuals against the reconstructed parent (eq. 3 with the pixel and
// block-energy thresholds and the quantiser, Sec. 3.2) run one thread per
// sample or per (node, block, channel); every group's bitmap, range codes
// and BISE payloads (Sec. 3.3-3.4) are packed by one thread per group after
// the host has turned the group sizes into offsets.  The host then writes
// the header, the raw top level and the offsets around the packed words.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "encode.h"
#include "internal.h"

namespace {

constexpr int kT = 256;

struct EncGeo {
  int U, V, W, H, wp, hp, B, S, L, q, nbx, nb, ng, n_srv, nbw;
  int lu[lfc::kMaxLevels], lv[lfc::kMaxLevels], c[lfc::kMaxLevels];
  int pix_thr, blk_thr;
};

// allowed BISE ranges by increasing number of values: (values, code)
struct RangeTab {
  int n;
  int bound[lfc::kNumCodes], code[lfc::kNumCodes];
};

__device__ __forceinline__ int32_t floor_div_d(int64_t x, int64_t d) {
  return (int32_t)(x >= 0 ? x / d : -((-x + d - 1) / d));
}

__device__ __forceinline__ uint32_t zz(int32_t v) { return (uint16_t)(((uint32_t)v << 1) ^ (uint32_t)(v >> 31)); }

// range code k: kind (0 bits, 1 trit, 2 quint) and low-bit count m
__device__ __forceinline__ void code_km(int k, int &kind, int &m) {
  if (k < 12) {
    kind = 0;
    m = k + 1;
  } else if (k < 19) {
    kind = 1;
    m = k - 12;
  } else {
    kind = 2;
    m = k - 19;
  }
}

__device__ __forceinline__ uint32_t block_bits_d(int k, int S) {
  int kind, m;
  code_km(k, kind, m);
  const uint32_t plane = kind == 1 ? (8u * S + 4u) / 5u : (kind == 2 ? (7u * S + 2u) / 3u : 0u);
  return (uint32_t)(S * m) + plane;
}

__device__ __forceinline__ void put_field_d(uint32_t *w, uint64_t pos, uint32_t v) {
  const uint64_t x = (uint64_t)v << (pos & 31);
  w[pos >> 5] |= (uint32_t)x;
  if (x >> 32) w[(pos >> 5) + 1] |= (uint32_t)(x >> 32);
}

// level 0: padded YCoCg-R planes [nv][3][hp][wp], edges replicated
__global__ __launch_bounds__(kT) void k_enc_level0(const uint8_t *rgb, int16_t *lvl, EncGeo g) {
  const int x = blockIdx.x * kT + threadIdx.x, y = blockIdx.y, vi = blockIdx.z;
  if (x >= g.wp) return;
  const int sx = min(x, g.W - 1), sy = min(y, g.H - 1);
  const uint8_t *px = rgb + (((size_t)vi * g.H + sy) * g.W + sx) * 3;
  const int co = px[0] - px[2];
  const int t = px[2] + (co >> 1);
  const int cg = px[1] - t;
  const size_t plane = (size_t)g.hp * g.wp, o = (size_t)vi * 3 * plane + (size_t)y * g.wp + x;
  lvl[o] = (int16_t)(t + (cg >> 1));
  lvl[o + plane] = (int16_t)co;
  lvl[o + 2 * plane] = (int16_t)cg;
}

// level l >= 1: the binomial-weighted, rounded mean of each cluster of
// level l-1 over the members that exist (eqs. 1-2)
__global__ __launch_bounds__(kT) void k_enc_filter(const int16_t *below, int16_t *above, EncGeo g, int l) {
  const int x = blockIdx.x * kT + threadIdx.x, y = blockIdx.y % g.hp, ch = blockIdx.y / g.hp, node = blockIdx.z;
  if (x >= g.wp) return;
  const int c = g.c[l], nx = node % g.lu[l], ny = node / g.lu[l];
  int64_t pascal[8] = {1, 0, 0, 0, 0, 0, 0, 0};
  for (int i = 1; i < c; i++)
    for (int k = i; k >= 1; k--) pascal[k] += pascal[k - 1];
  const size_t plane = (size_t)g.hp * g.wp, img = 3 * plane, off = (size_t)ch * plane + (size_t)y * g.wp + x;
  int64_t wsum = 0, acc = 0;
  for (int yy = ny * c; yy < min(ny * c + c, g.lv[l - 1]); yy++)
    for (int xx = nx * c; xx < min(nx * c + c, g.lu[l - 1]); xx++) {
      const int64_t w = pascal[xx - nx * c] * pascal[yy - ny * c];
      wsum += w;
      acc += w * below[(size_t)(yy * g.lu[l - 1] + xx) * img + off];
    }
  above[(size_t)node * img + off] = (int16_t)floor_div_d(acc + wsum / 2, wsum);
}

// one (node, block, channel) of level l: residual against the reconstructed
// parent, pixel threshold, block-energy threshold, quantiser, range code;
// writes the code table, the zigzag values and the reconstruction
__global__ __launch_bounds__(kT) void k_enc_residual(const int16_t *own_lvl, const int16_t *par_rec, int16_t *rec,
                                                     const int32_t *serial, int8_t *code_tab, uint16_t *zv,
                                                     int32_t *err, EncGeo g, RangeTab rt, int l) {
  const int64_t r = (int64_t)blockIdx.x * kT + threadIdx.x;
  const int nodes = g.lu[l] * g.lv[l];
  if (r >= (int64_t)nodes * g.nb * 3) return;
  const int ch = (int)(r % 3), b = (int)((r / 3) % g.nb), node = (int)(r / 3 / g.nb);
  const int cp = g.c[l + 1], nx = node % g.lu[l], ny = node / g.lu[l];
  const int parent = (ny / cp) * g.lu[l + 1] + nx / cp;
  const int bx = b % g.nbx, by = b / g.nbx, B = g.B, S = g.S;
  const size_t plane = (size_t)g.hp * g.wp, img = 3 * plane;
  const size_t base = (size_t)ch * plane + (size_t)by * B * g.wp + (size_t)bx * B;
  const int16_t *own = own_lvl + (size_t)node * img + base;
  const int16_t *par = par_rec + (size_t)parent * img + base;
  int16_t *dst = rec + (size_t)node * img + base;
  int32_t v[64];
  int64_t energy = 0;
  for (int i = 0; i < S; i++) {
    const size_t d = (size_t)(i / B) * g.wp + i % B;
    int32_t x = (int32_t)own[d] - (int32_t)par[d];
    if (abs(x) < g.pix_thr) x = 0;
    v[i] = x;
    energy += abs(x);
  }
  bool keep = energy > g.blk_thr;
  uint32_t zmax = 0;
  if (keep) {
    bool nz = false;
    for (int i = 0; i < S; i++) {
      if (g.q) {
        const int32_t mag = (abs(v[i]) + (1 << (g.q - 1))) >> g.q;
        v[i] = v[i] < 0 ? -mag : mag;
      }
      nz |= v[i] != 0;
      zmax = max(zmax, zz(v[i]));
    }
    keep = nz;
  }
  const size_t key = (size_t)(3 * b + ch) * g.n_srv + serial[node];
  int code = -1;
  if (keep) {
    for (int i = 0; i < rt.n; i++)
      if ((uint32_t)rt.bound[i] > zmax) {
        code = rt.code[i];
        break;
      }
    if (code < 0) {
      atomicOr(err, 1);
      return;
    }
    for (int i = 0; i < S; i++) zv[key * S + i] = (uint16_t)zz(v[i]);
  }
  code_tab[key] = (int8_t)code;
  for (int i = 0; i < S; i++) {
    const size_t d = (size_t)(i / B) * g.wp + i % B;
    const int32_t x = (int32_t)par[d] + (keep ? v[i] * (1 << g.q) : 0);
    if (x < -32768 || x > 32767) atomicOr(err, 2);
    dst[d] = (int16_t)x;
  }
}

// words of each group: bitmap, 5-bit codes, payload (0 for an empty group)
__global__ __launch_bounds__(kT) void k_enc_group_words(const int8_t *code_tab, uint32_t *gwords, EncGeo g) {
  const int gi = blockIdx.x * kT + threadIdx.x;
  if (gi >= g.ng) return;
  const int8_t *ct = code_tab + (size_t)gi * g.n_srv;
  uint64_t present = 0, bits = 0;
  for (int s = 0; s < g.n_srv; s++)
    if (ct[s] >= 0) {
      present++;
      bits += block_bits_d(ct[s], g.S);
    }
  gwords[gi] = present ? (uint32_t)(g.nbw + (5 * present + 31) / 32 + (bits + 31) / 32) : 0u;
}

// one group: bitmap, range codes in serial order, then the BISE payloads
// (digit plane, then the low-bit plane), into zeroed words at its offset
__global__ __launch_bounds__(kT) void k_enc_pack(const int8_t *code_tab, const uint16_t *zv, const uint32_t *offsets,
                                                 uint32_t *srv, EncGeo g) {
  const int gi = blockIdx.x * kT + threadIdx.x;
  if (gi >= g.ng || offsets[gi] == offsets[gi + 1]) return;
  uint32_t *w = srv + offsets[gi];
  const int8_t *ct = code_tab + (size_t)gi * g.n_srv;
  uint64_t present = 0;
  for (int s = 0; s < g.n_srv; s++)
    if (ct[s] >= 0) {
      w[s >> 5] |= 1u << (s & 31);
      present++;
    }
  uint64_t cpos = 32ull * g.nbw, pos = 32ull * (g.nbw + (5 * present + 31) / 32);
  const int S = g.S;
  for (int s = 0; s < g.n_srv; s++) {
    if (ct[s] < 0) continue;
    put_field_d(w, cpos, (uint32_t)ct[s]);
    cpos += 5;
    const uint16_t *z = zv + ((size_t)gi * g.n_srv + s) * S;
    int kind, m;
    code_km(ct[s], kind, m);
    if (kind) {
      const int glen = kind == 1 ? 5 : 3, radix = kind == 1 ? 3 : 5, full = kind == 1 ? 8 : 7;
      for (int i0 = 0; i0 < S; i0 += glen) {
        const int k = min(glen, S - i0);
        uint32_t num = 0;
        for (int rr = k - 1; rr >= 0; rr--) num = num * radix + (uint32_t)(z[i0 + rr] >> m);
        put_field_d(w, pos, num);
        pos += (full * k + glen - 1) / glen;
      }
    }
    const uint32_t lowmask = (1u << m) - 1u;
    for (int i = 0; i < S; i++, pos += m)
      if (m) put_field_d(w, pos, z[i] & lowmask);
  }
}

// the top level as the stream stores it: [n_top][nb][3][B*B]
__global__ __launch_bounds__(kT) void k_enc_top_blocks(const int16_t *top, int16_t *dst, EncGeo g, int n_top) {
  const int64_t r = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (r >= (int64_t)n_top * g.nb * 3 * g.S) return;
  const int i = (int)(r % g.S), ch = (int)((r / g.S) % 3), b = (int)((r / g.S / 3) % g.nb);
  const int n = (int)(r / g.S / 3 / g.nb), bx = b % g.nbx, by = b / g.nbx;
  const size_t plane = (size_t)g.hp * g.wp;
  dst[r] = top[(size_t)n * 3 * plane + (size_t)ch * plane + (size_t)(by * g.B + i / g.B) * g.wp + bx * g.B + i % g.B];
}

// squared error of every (view, channel) on the unpadded area: a workgroup
// sums kSseRows rows of one plane in registers, then across its waves, and
// adds once (one atomic per wave per row made the adds to a plane's counter
// queue behind each other)
constexpr int kSseRows = 64;
__global__ __launch_bounds__(kT) void k_enc_sse(const int16_t *rec0, const int16_t *lvl0, unsigned long long *sse,
                                                EncGeo g) {
  __shared__ unsigned long long part[kT / 64];
  const int vc = blockIdx.y, y0 = blockIdx.x * kSseRows, y1 = min(y0 + kSseRows, g.H);
  const size_t plane = (size_t)vc * g.hp * g.wp;
  int64_t e = 0;
  for (int y = y0; y < y1; y++)
    for (int x = threadIdx.x; x < g.W; x += kT) {
      const size_t o = plane + (size_t)y * g.wp + x;
      const int64_t d = (int64_t)rec0[o] - (int64_t)lvl0[o];
      e += d * d;
    }
  for (int off = 32; off > 0; off >>= 1) e += __shfl_down(e, off, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = (unsigned long long)e;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int w = 0; w < kT / 64; w++) t += part[w];
    if (t) atomicAdd(sse + vc, t);
  }
}

lfc_status launched(const char *what) {
  const hipError_t he = hipGetLastError();
  if (he != hipSuccess) return lfc::fail(LFC_E_HIP, std::string("lfc_encode_gpu: ") + what + ": " + hipGetErrorString(he));
  return LFC_OK;
}

// device buffers of one encode, freed on every path
struct DevBufs {
  std::vector<void *> ptrs;
  ~DevBufs() {
    for (void *p : ptrs) (void)hipFree(p);
  }
  template <typename T>
  lfc_status alloc(T **p, size_t n) {
    void *q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) {
      (void)hipGetLastError();
      return lfc::fail(LFC_E_NOMEM, "lfc_encode_gpu: device memory");
    }
    ptrs.push_back(q);
    *p = static_cast<T *>(q);
    return LFC_OK;
  }
};

}  // namespace

extern "C" lfc_status lfc_encode_gpu(const uint8_t *d_rgb, const lfc_params *p, void **stream_out, size_t *bytes_out,
                                     lfc_encode_stats *stats, hipStream_t s) {
  using namespace lfc;
  if (!d_rgb || !p || (!stream_out) != (!bytes_out)) return fail(LFC_E_INVALID, "lfc_encode_gpu: null argument");
  if (stream_out) {
    *stream_out = nullptr;
    *bytes_out = 0;
  }
  Geometry geo;
  std::string why;
  if (make_geometry(*p, geo, &why) != LFC_OK) return fail(LFC_E_INVALID, "lfc_encode_gpu: " + why);
  const int nv = geo.nv(), L = geo.L, S = geo.S;
  {
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    const size_t need = (size_t)nv * geo.H * geo.W * 3;
    if (hipMemGetAddressRange(&base, &size, const_cast<uint8_t *>(d_rgb)) != hipSuccess || !base ||
        (size_t)(d_rgb - static_cast<const uint8_t *>(base)) + need > size) {
      (void)hipGetLastError();
      return fail(LFC_E_INVALID, "lfc_encode_gpu: d_rgb is not device memory of [V][U][H][W][3] bytes");
    }
  }
  // grid limits of the launches below (second and third grid dimensions)
  bool fits = 3 * geo.hp <= 65535 && nv * 3 <= 65535;
  for (int l = 0; l < L; l++) fits &= geo.lu[l] * geo.lv[l] <= 65535;
  if (!fits) return fail(LFC_E_UNSUPPORTED, "lfc_encode_gpu: light field too large for the GPU encoder's grids");
  const uint32_t mask = p->range_mask ? p->range_mask : kAllCodes;
  EncGeo g{};
  g.U = geo.U, g.V = geo.V, g.W = geo.W, g.H = geo.H, g.wp = geo.wp, g.hp = geo.hp, g.B = geo.B, g.S = S, g.L = L;
  g.q = geo.q, g.nbx = geo.nbx, g.nb = geo.nb, g.ng = geo.ng, g.n_srv = geo.n_srv, g.nbw = geo.nbw;
  for (int l = 0; l < kMaxLevels; l++) g.lu[l] = geo.lu[l], g.lv[l] = geo.lv[l], g.c[l] = geo.c[l];
  g.pix_thr = p->pix_threshold, g.blk_thr = p->blk_threshold;
  RangeTab rt{};
  {
    std::vector<std::pair<int, int>> r;
    for (int k = 0; k < kNumCodes; k++)
      if ((mask >> k) & 1u) {
        const int bound = k < 12 ? 2 << k : (k < 19 ? 3 << (k - 12) : 5 << (k - 19));
        r.push_back({bound, k});
      }
    std::sort(r.begin(), r.end());
    rt.n = (int)r.size();
    for (int i = 0; i < rt.n; i++) rt.bound[i] = r[i].first, rt.code[i] = r[i].second;
  }
  TreeTables tt;
  try {
    build_tree_tables(geo, tt);
  } catch (const std::bad_alloc &) {
    return fail(LFC_E_NOMEM, "lfc_encode_gpu: out of host memory");
  }
  const size_t plane = (size_t)geo.hp * geo.wp, img = 3 * plane;
  const size_t nsg = (size_t)geo.ng * geo.n_srv;
  DevBufs db;
  std::vector<int16_t *> lvl(L, nullptr), rec(L, nullptr);
  std::vector<int32_t *> serial(L, nullptr);
  int8_t *code_tab = nullptr;
  uint16_t *zv = nullptr;
  int32_t *err = nullptr;
  uint32_t *gw = nullptr;
  for (int l = 0; l < L; l++) {
    const size_t nodes = (size_t)geo.lu[l] * geo.lv[l];
    if (lfc_status st = db.alloc(&lvl[l], nodes * img)) return st;
    if (l < L - 1) {
      if (lfc_status st = db.alloc(&rec[l], nodes * img)) return st;
      if (lfc_status st = db.alloc(&serial[l], nodes)) return st;
      if (hipMemcpyAsync(serial[l], tt.serial[l].data(), 4 * nodes, hipMemcpyHostToDevice, s) != hipSuccess)
        return fail(LFC_E_HIP, "lfc_encode_gpu: copy of the tree tables");
    }
  }
  rec[L - 1] = lvl[L - 1];   // the top level is stored losslessly
  if (lfc_status st = db.alloc(&code_tab, nsg)) return st;
  if (lfc_status st = db.alloc(&zv, nsg * S)) return st;
  if (lfc_status st = db.alloc(&err, 1)) return st;
  if (lfc_status st = db.alloc(&gw, (size_t)geo.ng)) return st;
  if (hipMemsetAsync(err, 0, 4, s) != hipSuccess || hipMemsetAsync(code_tab, 0xFF, std::max<size_t>(nsg, 1), s) != hipSuccess)
    return fail(LFC_E_HIP, "lfc_encode_gpu: clearing tables");

  // Stage I: level 0, then the key views of every level above
  hipLaunchKernelGGL(k_enc_level0, dim3((geo.wp + kT - 1) / kT, geo.hp, nv), dim3(kT), 0, s, d_rgb, lvl[0], g);
  if (lfc_status st = launched("level 0")) return st;
  for (int l = 1; l < L; l++) {
    hipLaunchKernelGGL(k_enc_filter, dim3((geo.wp + kT - 1) / kT, 3 * geo.hp, geo.lu[l] * geo.lv[l]), dim3(kT), 0, s,
                       (const int16_t *)lvl[l - 1], lvl[l], g, l);
    if (lfc_status st = launched("key-view filter")) return st;
  }
  // Stage II: residual levels from the top down against the reconstruction
  for (int l = L - 2; l >= 0; l--) {
    const int64_t rows = (int64_t)geo.lu[l] * geo.lv[l] * geo.nb * 3;
    hipLaunchKernelGGL(k_enc_residual, dim3((unsigned)((rows + kT - 1) / kT)), dim3(kT), 0, s,
                       (const int16_t *)lvl[l], (const int16_t *)rec[l + 1], rec[l], (const int32_t *)serial[l],
                       code_tab, zv, err, g, rt, l);
    if (lfc_status st = launched("residuals")) return st;
  }
  int32_t herr = 0;
  if (hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
    return fail(LFC_E_HIP, "lfc_encode_gpu: synchronize");
  if (herr & 1) return fail(LFC_E_RANGE, "lfc_encode_gpu: a residual block needs a BISE range the mask does not allow");
  if (herr & 2) return fail(LFC_E_RANGE, "lfc_encode_gpu: a reconstructed sample leaves int16");

  if (stats) {
    unsigned long long *sse = nullptr;
    if (lfc_status st = db.alloc(&sse, (size_t)nv * 3)) return st;
    if (hipMemsetAsync(sse, 0, 8ull * nv * 3, s) != hipSuccess) return fail(LFC_E_HIP, "lfc_encode_gpu: clearing");
    hipLaunchKernelGGL(k_enc_sse, dim3((geo.H + kSseRows - 1) / kSseRows, nv * 3), dim3(kT), 0, s,
                       (const int16_t *)(L > 1 ? rec[0] : lvl[0]), (const int16_t *)lvl[0], sse, g);
    if (lfc_status st = launched("squared error")) return st;
    std::vector<unsigned long long> hs((size_t)nv * 3);
    std::vector<int8_t> ct(std::max<size_t>(nsg, 1));
    if (hipMemcpyAsync(hs.data(), sse, 8ull * nv * 3, hipMemcpyDeviceToHost, s) != hipSuccess ||
        (nsg && hipMemcpyAsync(ct.data(), code_tab, nsg, hipMemcpyDeviceToHost, s) != hipSuccess) ||
        hipStreamSynchronize(s) != hipSuccess)
      return fail(LFC_E_HIP, "lfc_encode_gpu: copy of the statistics");
    std::vector<double> se(hs.begin(), hs.end());
    encode_stats_from_sse(se, nv, geo.W, geo.H, stats);
    std::fill(stats->code_hist, stats->code_hist + kNumCodes, 0);
    stats->present_blocks = 0;
    for (size_t i = 0; i < nsg; i++)
      if (ct[i] >= 0) {
        stats->code_hist[ct[i]]++;
        stats->present_blocks++;
      }
  }

  // Stage III: group sizes -> offsets (host) -> packed groups
  std::vector<uint32_t> gwords((size_t)geo.ng), offsets((size_t)geo.ng + 1);
  if (L > 1) {
    hipLaunchKernelGGL(k_enc_group_words, dim3((geo.ng + kT - 1) / kT), dim3(kT), 0, s, (const int8_t *)code_tab, gw, g);
    if (lfc_status st = launched("group sizes")) return st;
    if (hipMemcpyAsync(gwords.data(), gw, 4ull * geo.ng, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return fail(LFC_E_HIP, "lfc_encode_gpu: copy of the group sizes");
  }
  uint64_t acc = 0;
  for (int gi = 0; gi < geo.ng; gi++) {
    offsets[gi] = (uint32_t)acc;
    acc += gwords[gi];
    if (acc > 0xFFFFFFF0ull) return fail(LFC_E_RANGE, "lfc_encode_gpu: stream exceeds 2^32 words");
  }
  offsets[geo.ng] = (uint32_t)acc;
  const uint64_t srv_words = acc + 2;
  const uint64_t rkv_bytes = (uint64_t)geo.n_top * geo.nb * 3 * S * 2;
  const uint64_t rkv_off = kHeaderBytes, off_off = rkv_off + rkv_bytes, srv_off = off_off + 4ull * (geo.ng + 1);
  if (stats) stats->stream_bytes = srv_off + 4 * srv_words;
  if (!stream_out) return LFC_OK;
  uint32_t *d_off = nullptr, *d_srv = nullptr;
  int16_t *d_top = nullptr;
  if (lfc_status st = db.alloc(&d_off, (size_t)geo.ng + 1)) return st;
  if (lfc_status st = db.alloc(&d_srv, srv_words)) return st;
  if (lfc_status st = db.alloc(&d_top, rkv_bytes / 2)) return st;
  if (hipMemcpyAsync(d_off, offsets.data(), 4ull * (geo.ng + 1), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemsetAsync(d_srv, 0, 4 * srv_words, s) != hipSuccess)
    return fail(LFC_E_HIP, "lfc_encode_gpu: copy of the offsets");
  if (L > 1) {
    hipLaunchKernelGGL(k_enc_pack, dim3((geo.ng + kT - 1) / kT), dim3(kT), 0, s, (const int8_t *)code_tab,
                       (const uint16_t *)zv, (const uint32_t *)d_off, d_srv, g);
    if (lfc_status st = launched("packing")) return st;
  }
  const int64_t top_n = (int64_t)geo.n_top * geo.nb * 3 * S;
  hipLaunchKernelGGL(k_enc_top_blocks, dim3((unsigned)((top_n + kT - 1) / kT)), dim3(kT), 0, s,
                     (const int16_t *)lvl[L - 1], d_top, g, geo.n_top);
  if (lfc_status st = launched("top level")) return st;
  std::vector<uint8_t> out;
  try {
    out.assign(srv_off + 4 * srv_words, 0);
  } catch (const std::bad_alloc &) {
    return fail(LFC_E_NOMEM, "lfc_encode_gpu: out of host memory");
  }
  put_stream_header(out.data(), geo, *p, mask, rkv_off, off_off, srv_off);
  std::memcpy(out.data() + off_off, offsets.data(), 4ull * (geo.ng + 1));
  if (hipMemcpyAsync(out.data() + rkv_off, d_top, rkv_bytes, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(out.data() + srv_off, d_srv, 4 * srv_words, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(LFC_E_HIP, "lfc_encode_gpu: copy of the stream");
  void *mem = std::malloc(out.size());
  if (!mem) return fail(LFC_E_NOMEM, "lfc_encode_gpu: out of host memory");
  std::memcpy(mem, out.data(), out.size());
  *stream_out = mem;
  *bytes_out = out.size();
  return LFC_OK;
}

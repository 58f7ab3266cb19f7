// Host side of liblfc.so: parameters and geometry, the encoder (CompressLFI,
// Alg. 1) with its per-block control modes, the stream validator, decoder
// initialisation (Alg. 2 "Initialization"), which also builds the block
// directory used for random access and the whole-field kernel's strip
// tables, and the measured tuning of those tables.  See include/lfc.h for
// the contract of every exported call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <new>
#include <thread>

#include "encode.h"
#include "internal.h"

namespace lfc {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------

static thread_local std::string g_last_error;

lfc_status fail(lfc_status st, const std::string &msg) {
  g_last_error = msg;
  return st;
}

static std::string fmt(const char *f, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, f);
  vsnprintf(buf, sizeof buf, f, ap);
  va_end(ap);
  return buf;
}

// ---------------------------------------------------------------------------
// small parallel-for over [0, n) with a shared atomic cursor
// ---------------------------------------------------------------------------

static int worker_count() {
  unsigned hw = std::thread::hardware_concurrency();
  int n = hw ? (int)hw : 1;
  if (const char *e = getenv("OMP_NUM_THREADS")) {
    int v = atoi(e);
    if (v > 0) n = std::min(n, v);
  }
  return std::max(1, std::min(n, 16));
}

static void parallel_for(int64_t n, int64_t grain, const std::function<void(int64_t, int64_t)> &fn) {
  const int nt = worker_count();
  if (nt == 1 || n <= grain) {
    fn(0, n);
    return;
  }
  std::atomic<int64_t> next{0};
  auto work = [&] {
    for (;;) {
      int64_t a = next.fetch_add(grain);
      if (a >= n) break;
      fn(a, std::min(n, a + grain));
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < nt; t++) pool.emplace_back(work);
  work();
  for (auto &t : pool) t.join();
}

// ---------------------------------------------------------------------------
// geometry, range codes, tree
// ---------------------------------------------------------------------------

lfc_status make_geometry(const lfc_params &p, Geometry &g, std::string *why) {
  auto bad = [&](const std::string &m) {
    if (why) *why = m;
    return LFC_E_INVALID;
  };
  if (p.grid_u < 1 || p.grid_v < 1 || p.grid_u > 4096 || p.grid_v > 4096) return bad("grid_u/grid_v must be 1..4096");
  if (p.width < 1 || p.height < 1 || p.width > 65536 || p.height > 65536) return bad("width/height must be 1..65536");
  if (p.block != 2 && p.block != 4 && p.block != 8) return bad("block must be 2, 4 or 8");
  if (p.levels < 1 || p.levels > kMaxLevels) return bad("levels must be 1..6");
  if (p.pix_threshold < 0 || p.blk_threshold < 0) return bad("thresholds must be >= 0");
  if (p.quant_bits < 0 || p.quant_bits > 4) return bad("quant_bits must be 0..4");
  if (p.range_mask & ~kAllCodes) return bad("range_mask has bits above code 25");
  g = Geometry();
  g.U = p.grid_u;
  g.V = p.grid_v;
  g.W = p.width;
  g.H = p.height;
  g.B = p.block;
  g.S = p.block * p.block;
  g.L = p.levels;
  g.q = p.quant_bits;
  g.wp = (p.width + p.block - 1) / p.block * p.block;
  g.hp = (p.height + p.block - 1) / p.block * p.block;
  g.nbx = g.wp / g.B;
  g.nby = g.hp / g.B;
  if ((int64_t)g.nbx * g.nby * 3 > (int64_t)1 << 30) return bad("image too large");
  if ((int64_t)g.U * g.V * g.hp * g.wp * 3 > ((int64_t)1 << 40)) return bad("light field too large");
  g.nb = g.nbx * g.nby;
  g.ng = 3 * g.nb;
  g.lu[0] = g.U;
  g.lv[0] = g.V;
  for (int l = 1; l < g.L; l++) {
    int c = p.cluster[l - 1];
    if (c < 2 || c > 8) return bad("cluster sides must be 2..8");
    g.c[l] = c;
    g.lu[l] = (g.lu[l - 1] + c - 1) / c;
    g.lv[l] = (g.lv[l - 1] + c - 1) / c;
  }
  int64_t nsrv = 0;
  for (int l = 0; l + 1 < g.L; l++) nsrv += (int64_t)g.lu[l] * g.lv[l];
  if (nsrv > (1 << 20)) return bad("tree too large");
  g.n_srv = (int)nsrv;
  g.n_top = g.lu[g.L - 1] * g.lv[g.L - 1];
  g.nbw = (g.n_srv + 31) / 32;
  return LFC_OK;
}

// Range code k: 0..11 plain bits m = k+1; 12..18 trits m = k-12; 19..25
// quints m = k-19.  A block is the digit plane (one base-3 field per 5 values
// or base-5 field per 3 values) followed by S fields of m low bits.
struct RangeCode {
  int kind;    // 0 bits, 1 trit, 2 quint
  int m;
  int bound;   // number of representable values
};

static RangeCode range_code(int k) {
  if (k < 12) return {0, k + 1, 1 << (k + 1)};
  if (k < 19) return {1, k - 12, 3 << (k - 12)};
  return {2, k - 19, 5 << (k - 19)};
}

static int digit_plane_bits(int kind, int S) {
  if (kind == 1) return (8 * S + 4) / 5;   // ceil(8S/5): 5 trits in 8 bits
  if (kind == 2) return (7 * S + 2) / 3;   // ceil(7S/3): 3 quints in 7 bits
  return 0;
}

int bise_block_bits(int code, int S) {
  RangeCode r = range_code(code);
  return S * r.m + digit_plane_bits(r.kind, S);
}

// Breadth-first serial numbering of the tree (Sec. 3.4): the top-level nodes
// in row-major order, then, level by level, the children of each dequeued
// node in row-major order within its cluster.
void build_tree_tables(const Geometry &g, TreeTables &t) {
  const int L = g.L, nv = g.nv();
  t.serial.assign(L, {});
  for (int l = 0; l < L; l++) t.serial[l].assign((size_t)g.lu[l] * g.lv[l], -1);
  std::vector<std::pair<int, int>> fifo;
  fifo.reserve((size_t)g.n_srv + g.n_top);
  for (int i = 0; i < g.n_top; i++) fifo.push_back({L - 1, i});
  int32_t counter = 0;
  for (size_t head = 0; head < fifo.size(); head++) {
    auto [l, id] = fifo[head];
    if (l < L - 1) t.serial[l][id] = counter++;
    if (l == 0) continue;
    const int c = g.c[l], px = id % g.lu[l], py = id / g.lu[l];
    for (int yy = py * c; yy < std::min(py * c + c, g.lv[l - 1]); yy++)
      for (int xx = px * c; xx < std::min(px * c + c, g.lu[l - 1]); xx++)
        fifo.push_back({l - 1, yy * g.lu[l - 1] + xx});
  }
  const int depth = std::max(L - 1, 0), stride = std::max(depth, 1);
  t.path.assign((size_t)nv * stride, 0);
  t.root.assign(nv, 0);
  for (int vi = 0; vi < nv; vi++) {
    int x = vi % g.U, y = vi / g.U;
    for (int l = 0; l < L; l++) {
      if (l > 0) {
        x /= g.c[l];
        y /= g.c[l];
      }
      const int id = y * g.lu[l] + x;
      if (l < L - 1) t.path[(size_t)vi * stride + l] = t.serial[l][id];
      else t.root[vi] = id;
    }
  }
  // runs of sibling leaves in serial order
  std::vector<int32_t> order(nv);
  for (int vi = 0; vi < nv; vi++) order[vi] = vi;
  if (L > 1)
    std::sort(order.begin(), order.end(),
              [&](int a, int b) { return t.path[(size_t)a * stride] < t.path[(size_t)b * stride]; });
  auto same_ancestors = [&](int a, int b) {
    if (t.root[a] != t.root[b]) return false;
    for (int l = 1; l < L - 1; l++)
      if (t.path[(size_t)a * stride + l] != t.path[(size_t)b * stride + l]) return false;
    return L > 1;
  };
  t.batch.clear();
  for (int k = 0; k < nv;) {
    int n = 1;
    while (n < kBatch && k + n < nv && same_ancestors(order[k], order[k + n])) n++;
    int32_t rec[kBatchWords];
    for (int i = 0; i < kBatchWords; i++) rec[i] = (i >= 1 && i <= 9) ? -1 : 0;
    rec[0] = n;
    for (int i = 0; i < n; i++) rec[1 + i] = order[k + i];
    const int v0 = order[k];
    rec[5] = t.root[v0];
    for (int l = L - 2, i = 0; l >= 1; l--, i++) rec[6 + i] = t.path[(size_t)v0 * stride + l];
    rec[10] = L > 1 ? t.path[(size_t)v0 * stride] : -1;
    t.batch.insert(t.batch.end(), rec, rec + kBatchWords);
    k += n;
  }
}

// Decode schedule of the whole-field kernel, derived once from the directory.
// Per strip (channel c, block row by, strip sx of 64/B blocks) the runs of
// sibling leaves are cut into chunks whose stored blocks fit the kernel's
// compact residual tile (cap blocks, stored blocks only) and whose gather
// table (masks, first slots, run records) fits kLFTabWords words; per
// chunk: its runs, its nodes (leaves first, then ancestors), per node a mask
// of the stored blocks and the tile slot of the first one (slots follow node
// order, then block order), per run the positions of its first leaf and of
// its ancestors in the node list, and the stored blocks sorted by range kind
// with their directory entries and (slot << 5 | block).
//   strip record: [0] chunks, [1..chunks] chunk record offsets from the
//   strip's start, [chunks+1] the strip's length;
//   chunk record: q0, nq, nn, n0, n01, n (first run, runs, nodes, ends of the
//   plain-bit, trit and quint blocks), masks[nn], first slots[nn] (16-bit, two
//   per word), runs[nq][3 words] (16-bit: first leaf, ancestors on levels
//   L-2 .. 1; 0xFFFF unused), entries[n], items[n] (16-bit, two per word).
static void build_schedule(const Geometry &g, const std::vector<uint32_t> &off, const std::vector<uint32_t> &srv,
                           const std::vector<uint32_t> &dbase, const std::vector<uint32_t> &poff,
                           const std::vector<int32_t> &batch, std::vector<uint32_t> &sched,
                           std::vector<uint32_t> &strip_off, int cap) {
  const int nblk = 64 / g.B, nsx = (g.nbx + nblk - 1) / nblk, nstrip = 3 * g.nby * nsx;
  const int nruns = (int)(batch.size() / kBatchWords), L = g.L;
  std::vector<std::vector<uint32_t>> per((size_t)nstrip);
  parallel_for(nstrip, 8, [&](int64_t a, int64_t e) {
    std::vector<uint32_t> m((size_t)std::max(g.n_srv, 1));
    std::vector<int> loc((size_t)std::max(g.n_srv, 1), -1);
    for (int64_t st = a; st < e; st++) {
      const int sx = (int)(st % nsx), by = (int)((st / nsx) % g.nby), c = (int)(st / ((int64_t)nsx * g.nby));
      // stored blocks of every node in this strip
      std::fill(m.begin(), m.end(), 0u);
      for (int jj = 0; jj < nblk; jj++) {
        const int bx = sx * nblk + jj;
        if (bx >= g.nbx) continue;
        const size_t gi = 3 * ((size_t)by * g.nbx + bx) + c;
        if (off[gi] == off[gi + 1]) continue;
        for (int w = 0; w < g.nbw; w++)
          for (uint32_t bm = srv[off[gi] + w]; bm; bm &= bm - 1) m[(size_t)w * 32 + __builtin_ctz(bm)] |= 1u << jj;
      }
      std::vector<uint32_t> head(1, 0), body;
      for (int q = 0; q < nruns;) {
        // greedy: consecutive runs while their nodes' stored blocks fit the tile
        std::vector<int> leaves, ancs;
        int count = 0, k = 0;
        while (q + k < nruns) {
          const int32_t *r = &batch[(size_t)(q + k) * kBatchWords];
          int add = 0;
          std::vector<int> nl, na;
          for (int i = 0; i < r[0] && L > 1; i++) {   // (a tree of height 1 has no residual nodes)
            const int s = r[10] + i;
            if (loc[(size_t)s] < 0) {
              nl.push_back(s);
              add += __builtin_popcount(m[(size_t)s]);
            }
          }
          for (int i = 0; i < L - 2; i++) {
            const int s = r[6 + i];
            if (loc[(size_t)s] < 0 && std::find(na.begin(), na.end(), s) == na.end()) {
              na.push_back(s);
              add += __builtin_popcount(m[(size_t)s]);
            }
          }
          const size_t nn_new = leaves.size() + ancs.size() + nl.size() + na.size();
          if (k > 0 && (count + add > cap || nn_new + (nn_new + 1) / 2 + 3 * (size_t)(k + 1) > (size_t)kLFTabWords))
            break;
          for (int s : nl) {
            loc[(size_t)s] = 0;
            leaves.push_back(s);
          }
          for (int s : na) {
            loc[(size_t)s] = 0;
            ancs.push_back(s);
          }
          count += add;
          k++;
        }
        // local node order: leaves, then ancestors
        std::vector<int> nodes(leaves);
        nodes.insert(nodes.end(), ancs.begin(), ancs.end());
        for (size_t i = 0; i < nodes.size(); i++) loc[(size_t)nodes[i]] = (int)i;
        const int nn = (int)nodes.size();
        std::vector<uint32_t> masks((size_t)nn), bases((size_t)nn);
        uint32_t slot = 0;
        for (int i = 0; i < nn; i++) {
          masks[(size_t)i] = m[(size_t)nodes[(size_t)i]];
          bases[(size_t)i] = slot;
          slot += (uint32_t)__builtin_popcount(masks[(size_t)i]);
        }
        std::vector<uint32_t> ent[3], item[3];
        for (int i = 0; i < nn; i++) {
          const int s = nodes[(size_t)i];
          for (uint32_t bits = masks[(size_t)i]; bits; bits &= bits - 1) {
            const int jj = __builtin_ctz(bits);
            const size_t gi = 3 * ((size_t)by * g.nbx + sx * nblk + jj) + c;
            const uint32_t bm = srv[off[gi] + (s >> 5)], bit = (uint32_t)s & 31u;
            const uint32_t en = poff[dbase[gi * g.nbw + (s >> 5)] + (uint32_t)__builtin_popcount(bm & ((1u << bit) - 1u))];
            const uint32_t code = en & 31u;
            const int kind = code < 12 ? 0 : (code < 19 ? 1 : 2);
            const uint32_t sl = bases[(size_t)i] + (uint32_t)__builtin_popcount(masks[(size_t)i] & ((1u << jj) - 1u));
            ent[kind].push_back(en);
            item[kind].push_back((sl << 5) | (uint32_t)jj);
          }
        }
        const uint32_t n0 = (uint32_t)ent[0].size(), n01 = n0 + (uint32_t)ent[1].size();
        const uint32_t n = n01 + (uint32_t)ent[2].size();
        head.push_back((uint32_t)body.size());   // made absolute below
        body.push_back((uint32_t)q);
        body.push_back((uint32_t)k);
        body.push_back((uint32_t)nn);
        body.push_back(n0);
        body.push_back(n01);
        body.push_back(n);
        body.insert(body.end(), masks.begin(), masks.end());
        for (int i = 0; i < nn; i += 2)
          body.push_back(bases[(size_t)i] | (i + 1 < nn ? bases[(size_t)i + 1] << 16 : 0u));
        for (int j = 0; j < k; j++) {
          const int32_t *r = &batch[(size_t)(q + j) * kBatchWords];
          uint32_t h[4] = {L > 1 ? (uint32_t)loc[(size_t)r[10]] : 0xFFFFu, 0xFFFFu, 0xFFFFu, 0xFFFFu};
          for (int i = 0; i < std::min(L - 2, 3); i++) h[1 + i] = (uint32_t)loc[(size_t)r[6 + i]];
          body.push_back(h[0] | (h[1] << 16));
          body.push_back(h[2] | (h[3] << 16));
          body.push_back(L - 2 > 3 ? (uint32_t)loc[(size_t)r[9]] | 0xFFFF0000u : 0xFFFFFFFFu);
        }
        for (int kind = 0; kind < 3; kind++) body.insert(body.end(), ent[kind].begin(), ent[kind].end());
        std::vector<uint32_t> all;
        for (int kind = 0; kind < 3; kind++) all.insert(all.end(), item[kind].begin(), item[kind].end());
        for (size_t i = 0; i < all.size(); i += 2) body.push_back(all[i] | (i + 1 < all.size() ? all[i + 1] << 16 : 0u));
        for (int s : nodes) loc[(size_t)s] = -1;
        q += k;
      }
      const uint32_t nck = (uint32_t)(head.size() - 1);
      head[0] = nck;
      const uint32_t hdr = nck + 2;
      for (uint32_t i = 1; i <= nck; i++) head[i] += hdr;
      head.push_back(hdr + (uint32_t)body.size());
      std::vector<uint32_t> &w = per[(size_t)st];
      w = head;
      w.insert(w.end(), body.begin(), body.end());
    }
  });
  strip_off.assign((size_t)nstrip + 1, 0);
  size_t total = 0;
  for (int st = 0; st < nstrip; st++) {
    strip_off[(size_t)st] = (uint32_t)total;
    total += per[(size_t)st].size();
  }
  strip_off[(size_t)nstrip] = (uint32_t)total;
  sched.resize(total);
  for (int st = 0; st < nstrip; st++) std::copy(per[(size_t)st].begin(), per[(size_t)st].end(), sched.begin() + strip_off[(size_t)st]);
}

// Decode schedule of the colour whole-field kernel, which writes each pixel
// as 8-bit RGB and so needs a pixel's three channels in one workgroup: a
// strip (block row by, strip sx of 64/B blocks) covers all three channels,
// and its chunks count the stored blocks of the three channels against the
// tile capacity.  Otherwise as build_schedule:
//   strip record: [0] chunks, [1..chunks] chunk record offsets from the
//   strip's start, [chunks+1] the strip's length;
//   chunk record: q0, nq, nn, n0, n01, n, masks[3][nn] (channel-major),
//   first slots[3][nn] (16-bit, two per word), runs[nq][3 words],
//   entries[n], items[n] (32-bit: slot << 20 | node << 8 | channel << 6 |
//   block; a chunk has at most kRGBNodeCap nodes and kRGBNodeCap runs).
static void build_schedule_rgb(const Geometry &g, const std::vector<uint32_t> &off, const std::vector<uint32_t> &srv,
                               const std::vector<uint32_t> &dbase, const std::vector<uint32_t> &poff,
                               const std::vector<int32_t> &batch, std::vector<uint32_t> &sched,
                               std::vector<uint32_t> &strip_off, int cap) {
  const int nblk = 64 / g.B, nsx = (g.nbx + nblk - 1) / nblk, nstrip = g.nby * nsx;
  const int nruns = (int)(batch.size() / kBatchWords), L = g.L;
  const size_t ns = (size_t)std::max(g.n_srv, 1);
  std::vector<std::vector<uint32_t>> per((size_t)nstrip);
  parallel_for(nstrip, 8, [&](int64_t a, int64_t e) {
    std::vector<uint32_t> m(3 * ns);   // [channel][node] stored-block mask of the strip
    std::vector<int> loc(ns, -1);
    for (int64_t st = a; st < e; st++) {
      const int sx = (int)(st % nsx), by = (int)(st / nsx);
      std::fill(m.begin(), m.end(), 0u);
      for (int c = 0; c < 3; c++)
        for (int jj = 0; jj < nblk; jj++) {
          const int bx = sx * nblk + jj;
          if (bx >= g.nbx) continue;
          const size_t gi = 3 * ((size_t)by * g.nbx + bx) + c;
          if (off[gi] == off[gi + 1]) continue;
          for (int w = 0; w < g.nbw; w++)
            for (uint32_t bm = srv[off[gi] + w]; bm; bm &= bm - 1)
              m[c * ns + (size_t)w * 32 + __builtin_ctz(bm)] |= 1u << jj;
        }
      auto stored = [&](int s) {
        return __builtin_popcount(m[(size_t)s]) + __builtin_popcount(m[ns + (size_t)s]) +
               __builtin_popcount(m[2 * ns + (size_t)s]);
      };
      std::vector<uint32_t> head(1, 0), body;
      for (int q = 0; q < nruns;) {
        // greedy: consecutive runs while their nodes' stored blocks fit the tile
        std::vector<int> leaves, ancs;
        int count = 0, k = 0;
        while (q + k < nruns) {
          const int32_t *r = &batch[(size_t)(q + k) * kBatchWords];
          int add = 0;
          std::vector<int> nl, na;
          for (int i = 0; i < r[0] && L > 1; i++) {
            const int s = r[10] + i;
            if (loc[(size_t)s] < 0) {
              nl.push_back(s);
              add += stored(s);
            }
          }
          for (int i = 0; i < L - 2; i++) {
            const int s = r[6 + i];
            if (loc[(size_t)s] < 0 && std::find(na.begin(), na.end(), s) == na.end()) {
              na.push_back(s);
              add += stored(s);
            }
          }
          if (k > 0 && (count + add > cap || k >= kRGBNodeCap ||
                        leaves.size() + ancs.size() + nl.size() + na.size() > (size_t)kRGBNodeCap))
            break;
          for (int s : nl) {
            loc[(size_t)s] = 0;
            leaves.push_back(s);
          }
          for (int s : na) {
            loc[(size_t)s] = 0;
            ancs.push_back(s);
          }
          count += add;
          k++;
        }
        std::vector<int> nodes(leaves);
        nodes.insert(nodes.end(), ancs.begin(), ancs.end());
        for (size_t i = 0; i < nodes.size(); i++) loc[(size_t)nodes[i]] = (int)i;
        const int nn = (int)nodes.size();
        std::vector<uint32_t> masks(3 * (size_t)nn), bases(3 * (size_t)nn);
        uint32_t slot = 0;
        for (int c = 0; c < 3; c++)
          for (int i = 0; i < nn; i++) {
            masks[(size_t)c * nn + i] = m[c * ns + (size_t)nodes[(size_t)i]];
            bases[(size_t)c * nn + i] = slot;
            slot += (uint32_t)__builtin_popcount(masks[(size_t)c * nn + i]);
          }
        std::vector<uint32_t> ent[3], item[3];
        for (int c = 0; c < 3; c++)
          for (int i = 0; i < nn; i++) {
            const int s = nodes[(size_t)i];
            const uint32_t mk = masks[(size_t)c * nn + i];
            for (uint32_t bits = mk; bits; bits &= bits - 1) {
              const int jj = __builtin_ctz(bits);
              const size_t gi = 3 * ((size_t)by * g.nbx + sx * nblk + jj) + c;
              const uint32_t bm = srv[off[gi] + (s >> 5)], bit = (uint32_t)s & 31u;
              const uint32_t en =
                  poff[dbase[gi * g.nbw + (s >> 5)] + (uint32_t)__builtin_popcount(bm & ((1u << bit) - 1u))];
              const uint32_t code = en & 31u;
              const int kind = code < 12 ? 0 : (code < 19 ? 1 : 2);
              const uint32_t sl = bases[(size_t)c * nn + i] + (uint32_t)__builtin_popcount(mk & ((1u << jj) - 1u));
              ent[kind].push_back(en);
              item[kind].push_back((sl << 20) | ((uint32_t)i << 8) | ((uint32_t)c << 6) | (uint32_t)jj);
            }
          }
        const uint32_t n0 = (uint32_t)ent[0].size(), n01 = n0 + (uint32_t)ent[1].size();
        const uint32_t n = n01 + (uint32_t)ent[2].size();
        head.push_back((uint32_t)body.size());   // made absolute below
        body.push_back((uint32_t)q);
        body.push_back((uint32_t)k);
        body.push_back((uint32_t)nn);
        body.push_back(n0);
        body.push_back(n01);
        body.push_back(n);
        body.insert(body.end(), masks.begin(), masks.end());
        for (int i = 0; i < 3 * nn; i += 2)
          body.push_back(bases[(size_t)i] | (i + 1 < 3 * nn ? bases[(size_t)i + 1] << 16 : 0u));
        for (int j = 0; j < k; j++) {
          const int32_t *r = &batch[(size_t)(q + j) * kBatchWords];
          uint32_t h[4] = {L > 1 ? (uint32_t)loc[(size_t)r[10]] : 0xFFFFu, 0xFFFFu, 0xFFFFu, 0xFFFFu};
          for (int i = 0; i < std::min(L - 2, 3); i++) h[1 + i] = (uint32_t)loc[(size_t)r[6 + i]];
          body.push_back(h[0] | (h[1] << 16));
          body.push_back(h[2] | (h[3] << 16));
          body.push_back(L - 2 > 3 ? (uint32_t)loc[(size_t)r[9]] | 0xFFFF0000u : 0xFFFFFFFFu);
        }
        for (int kind = 0; kind < 3; kind++) body.insert(body.end(), ent[kind].begin(), ent[kind].end());
        for (int kind = 0; kind < 3; kind++) body.insert(body.end(), item[kind].begin(), item[kind].end());
        for (int s : nodes) loc[(size_t)s] = -1;
        q += k;
      }
      const uint32_t nck = (uint32_t)(head.size() - 1);
      head[0] = nck;
      const uint32_t hdr = nck + 2;
      for (uint32_t i = 1; i <= nck; i++) head[i] += hdr;
      head.push_back(hdr + (uint32_t)body.size());
      std::vector<uint32_t> &w = per[(size_t)st];
      w = head;
      w.insert(w.end(), body.begin(), body.end());
    }
  });
  strip_off.assign((size_t)nstrip + 1, 0);
  size_t total = 0;
  for (int st = 0; st < nstrip; st++) {
    strip_off[(size_t)st] = (uint32_t)total;
    total += per[(size_t)st].size();
  }
  strip_off[(size_t)nstrip] = (uint32_t)total;
  sched.resize(total);
  for (int st = 0; st < nstrip; st++) std::copy(per[(size_t)st].begin(), per[(size_t)st].end(), sched.begin() + strip_off[(size_t)st]);
}

// Everything the whole-field kernel needs per strip for one tile capacity:
// the decode schedule, the order in which workgroups take the strips
// (costliest first, staged words as the cost, so that short strips fill the
// tail of the launch), and per strip the LDS words of groups + schedule and
// of the schedule alone.
struct StripTables {
  std::vector<uint32_t> sched, strip_off, order, need;
  uint32_t max_words = 0;
};

static void make_strip_tables(const Geometry &g, const std::vector<uint32_t> &off, const std::vector<uint32_t> &srv,
                              const std::vector<uint32_t> &dbase, const std::vector<uint32_t> &poff,
                              const std::vector<int32_t> &batch, int cap, StripTables &t) {
  build_schedule(g, off, srv, dbase, poff, batch, t.sched, t.strip_off, cap);
  const int nblk = 64 / g.B, nsx = (g.nbx + nblk - 1) / nblk;
  const size_t nst = t.strip_off.size() - 1;
  std::vector<uint64_t> cost(nst);
  t.need.assign(2 * nst, 0);
  t.max_words = 0;
  for (size_t st = 0; st < nst; st++) {
    const int sx = (int)(st % nsx), by = (int)((st / nsx) % g.nby), c = (int)(st / ((size_t)nsx * g.nby));
    const uint64_t sw = t.strip_off[st + 1] - t.strip_off[st];
    uint64_t w = sw;
    for (int bx = sx * nblk; bx < std::min(sx * nblk + nblk, g.nbx); bx++) {
      const size_t gi = 3 * ((size_t)by * g.nbx + bx) + c;
      w += off[gi + 1] - off[gi];
    }
    cost[st] = w;
    t.need[2 * st] = (uint32_t)std::min<uint64_t>(w, 1u << 30);
    t.need[2 * st + 1] = (uint32_t)sw;
    t.max_words = std::max(t.max_words, t.need[2 * st]);
  }
  std::vector<uint32_t> perm(nst);
  for (size_t i = 0; i < nst; i++) perm[i] = (uint32_t)i;
  std::stable_sort(perm.begin(), perm.end(), [&](uint32_t x, uint32_t y) { return cost[x] > cost[y]; });
  // one order entry per workgroup (order_words): strip, schedule start and
  // length, then the strip's group starts and lengths
  const int ow = order_words(g.B);
  t.order.assign(nst * (size_t)ow, 0u);
  for (size_t i = 0; i < nst; i++) {
    const uint32_t st = perm[i];
    uint32_t *e = &t.order[i * (size_t)ow];
    const int sx = (int)(st % nsx), by = (int)((st / nsx) % g.nby), c = (int)(st / ((size_t)nsx * g.nby));
    e[0] = st;
    e[1] = t.strip_off[st];
    e[2] = t.strip_off[st + 1] - t.strip_off[st];
    for (int j = 0; j < nblk; j++) {
      const int bx = sx * nblk + j;
      if (bx >= g.nbx) continue;
      const size_t gi = 3 * ((size_t)by * g.nbx + bx) + c;
      e[4 + j] = off[gi];
      e[4 + nblk + j] = off[gi + 1] - off[gi];
    }
  }
}

// The colour kernel's strip tables: schedule and the order in which
// workgroups take the strips (costliest first: schedule words plus the
// strip's group words of all three channels).
static void make_strip_tables_rgb(const Geometry &g, const std::vector<uint32_t> &off, const std::vector<uint32_t> &srv,
                                  const std::vector<uint32_t> &dbase, const std::vector<uint32_t> &poff,
                                  const std::vector<int32_t> &batch, int cap, StripTables &t) {
  build_schedule_rgb(g, off, srv, dbase, poff, batch, t.sched, t.strip_off, cap);
  const int nblk = 64 / g.B, nsx = (g.nbx + nblk - 1) / nblk;
  const size_t nst = t.strip_off.size() - 1;
  std::vector<uint64_t> cost(nst);
  t.need.clear();
  t.max_words = 0;
  for (size_t st = 0; st < nst; st++) {
    const int sx = (int)(st % nsx), by = (int)(st / nsx);
    uint64_t w = t.strip_off[st + 1] - t.strip_off[st];
    for (int bx = sx * nblk; bx < std::min(sx * nblk + nblk, g.nbx); bx++)
      for (int c = 0; c < 3; c++) {
        const size_t gi = 3 * ((size_t)by * g.nbx + bx) + c;
        w += off[gi + 1] - off[gi];
      }
    cost[st] = w;
  }
  t.order.resize(nst);
  for (size_t i = 0; i < nst; i++) t.order[i] = (uint32_t)i;
  std::stable_sort(t.order.begin(), t.order.end(), [&](uint32_t x, uint32_t y) { return cost[x] > cost[y]; });
}

// ---------------------------------------------------------------------------
// encoder
// ---------------------------------------------------------------------------

// ORs a value of at most 32 bits into a zeroed word array at bit position pos.
static inline void put_field(uint32_t *w, uint64_t pos, uint32_t v) {
  const uint64_t x = (uint64_t)v << (pos & 31);
  w[pos >> 5] |= (uint32_t)x;
  if (x >> 32) w[(pos >> 5) + 1] |= (uint32_t)(x >> 32);
}

static inline int32_t floor_div(int64_t x, int64_t d) {
  return (int32_t)(x >= 0 ? x / d : -((-x + d - 1) / d));
}

static inline uint16_t zz_encode(int32_t v) { return (uint16_t)(((uint32_t)v << 1) ^ (uint32_t)(v >> 31)); }

// BISE packing of one block (Sec. 3.3): digit plane, then low-bit plane.
static uint64_t pack_block(uint32_t *w, uint64_t pos, const uint16_t *z, int S, int code) {
  const RangeCode rc = range_code(code);
  if (rc.kind) {
    const int glen = rc.kind == 1 ? 5 : 3, radix = rc.kind == 1 ? 3 : 5, full = rc.kind == 1 ? 8 : 7;
    for (int i0 = 0; i0 < S; i0 += glen) {
      const int k = std::min(glen, S - i0);
      uint32_t num = 0;
      for (int r = k - 1; r >= 0; r--) num = num * radix + (uint32_t)(z[i0 + r] >> rc.m);
      put_field(w, pos, num);
      pos += (full * k + glen - 1) / glen;
    }
  }
  const uint32_t lowmask = (1u << rc.m) - 1u;
  for (int i = 0; i < S; i++, pos += rc.m)
    if (rc.m) put_field(w, pos, z[i] & lowmask);
  return pos;
}

void put_stream_header(uint8_t *h, const Geometry &g, const lfc_params &p, uint32_t mask, uint64_t rkv_off,
                       uint64_t off_off, uint64_t srv_off) {
  std::memset(h, 0, kHeaderBytes);
  std::memcpy(h, "RLFC", 4);
  const uint16_t ver[2] = {1, (uint16_t)kHeaderBytes};
  std::memcpy(h + 4, ver, 4);
  int32_t f[23] = {g.U, g.V, g.W, g.H, g.wp, g.hp, g.B, g.L, g.q, 3, 0, 0, 0, 0, 0, 0,
                   p.pix_threshold, p.blk_threshold, (int32_t)mask, g.n_srv, g.n_top, g.nb, g.ng};
  for (int l = 1; l < g.L; l++) f[10 + l - 1] = g.c[l];
  std::memcpy(h + 8, f, sizeof f);
  const uint64_t o[3] = {rkv_off, off_off, srv_off};
  std::memcpy(h + 104, o, sizeof o);
}

void encode_stats_from_sse(const std::vector<double> &se, int nv, int W, int H, lfc_encode_stats *stats) {
  std::vector<double> ps(se.size());
  for (size_t r = 0; r < se.size(); r++) {
    const double mse = se[r] / ((double)W * H);
    ps[r] = mse > 0 ? std::min(100.0, 10.0 * std::log10(255.0 * 255.0 / mse)) : 100.0;
  }
  double sy = 0, sco = 0, scg = 0, sall = 0;
  for (int vi = 0; vi < nv; vi++) {
    sy += ps[3 * vi];
    sco += ps[3 * vi + 1];
    scg += ps[3 * vi + 2];
    sall += (6 * ps[3 * vi] + ps[3 * vi + 1] + ps[3 * vi + 2]) / 8;
  }
  stats->psnr = sall / nv;
  stats->psnr_y = sy / nv;
  stats->psnr_co = sco / nv;
  stats->psnr_cg = scg / nv;
}

// Per-block encoder control (learned encoder control; the paper applies one
// pixel threshold and one block-energy threshold to every block, Sec. 3.2).
// A block's options are the threshold classes: a pixel threshold from
// kCtlTau (then quantisation, the block stored if any value is nonzero), or
// dropping the block.
static const int kCtlTau[LFC_CTL_CLASSES - 1] = {0, 2, 3, 4, 5, 6, 8, 12, 16};

struct Candidate {
  int32_t qv[64];   // quantised values
  int code;         // range code, -1 absent
  int64_t sse;      // squared error of the reconstruction against the block
  int64_t rate;     // 5-bit range code + BISE payload bits, 0 when absent
  bool ok;          // reconstruction stays in int16 and a range holds the values
};

static inline int32_t quantize_sample(int32_t v, int q) {
  if (!q) return v;
  const int32_t mag = (std::abs(v) + (1 << (q - 1))) >> q;
  return v < 0 ? -mag : mag;
}

// Threshold class k applied to residuals v (own - parent) of one block; with
// `rng` >= 0 the values are clamped into that range code's bound and it is
// used as the block's code; with rng < 0 the smallest allowed range holding
// the values is chosen.
static void apply_class(const int32_t *v, const int32_t *own, const int32_t *par, int S, int q, int k, int rng,
                        const std::vector<std::pair<int, int>> &ranges, Candidate &cd) {
  cd.code = -1;
  cd.ok = true;
  cd.rate = 0;
  bool any = false;
  if (k == LFC_CTL_DROP || rng == LFC_CTL_ABSENT) {
    for (int i = 0; i < S; i++) cd.qv[i] = 0;
  } else {
    const int tau = kCtlTau[k];
    int32_t lo = INT32_MIN, hi = INT32_MAX;
    if (rng >= 0) {
      const int bound = range_code(rng).bound;
      lo = -(bound / 2);
      hi = (bound - 1) / 2;
    }
    uint32_t zmax = 0;
    for (int i = 0; i < S; i++) {
      int32_t x = std::abs(v[i]) < tau ? 0 : v[i];
      x = std::min(std::max(quantize_sample(x, q), lo), hi);
      cd.qv[i] = x;
      any |= x != 0;
      zmax = std::max<uint32_t>(zmax, zz_encode(x));
    }
    if (any) {
      if (rng >= 0) {
        cd.code = rng;
      } else {
        for (const auto &rg : ranges)
          if ((uint32_t)rg.first > zmax) {
            cd.code = rg.second;
            break;
          }
        if (cd.code < 0) cd.ok = false;
      }
    }
  }
  if (cd.code < 0)
    for (int i = 0; i < S; i++) cd.qv[i] = 0;
  else
    cd.rate = 5 + bise_block_bits(cd.code, S);
  cd.sse = 0;
  for (int i = 0; i < S; i++) {
    const int32_t r = par[i] + (cd.code >= 0 ? cd.qv[i] * (1 << q) : 0);
    if (r < -32768 || r > 32767) cd.ok = false;
    const int64_t d = (int64_t)own[i] - r;
    cd.sse += d * d;
  }
}

// Exhaustive search: the class of least cost w_c * SSE * 2^16 + lambda_q16 *
// rate (w = 6 for Y, 1 for Co and Cg, the channel weights of eq. 4), ties to
// the lower class.  Returns the class; cd holds its candidate.
static int search_class(const int32_t *v, const int32_t *own, const int32_t *par, int S, int q, int ch,
                        int64_t lambda_q16, const std::vector<std::pair<int, int>> &ranges, Candidate &cd) {
  const int64_t wc = ch == 0 ? 6 : 1;
  int best = -1;
  int64_t bestj = 0;
  Candidate tmp;
  for (int k = 0; k < LFC_CTL_CLASSES; k++) {
    apply_class(v, own, par, S, q, k, -1, ranges, tmp);
    if (!tmp.ok) continue;
    const int64_t j = wc * tmp.sse * 65536 + lambda_q16 * tmp.rate;
    if (best < 0 || j < bestj) {
      best = k;
      bestj = j;
      cd = tmp;
    }
  }
  return best;   // LFC_CTL_DROP is always valid
}

// The 16 features of a block's decision (row-major B x B blocks): v the
// residuals, par the parent's reconstruction.
static void block_features(const int32_t *v, const int32_t *par, int B, int level, int ch, int q,
                           int64_t lambda_q16, float *f) {
  const int S = B * B;
  double sa = 0, sa2 = 0, amax = 0, c2 = 0, c4 = 0, c8 = 0, c16 = 0;
  double sp = 0, sp2 = 0, gx = 0, gy = 0, gmax = 0;
  for (int i = 0; i < S; i++) {
    const double a = std::abs(v[i]);
    sa += a;
    sa2 += a * a;
    amax = std::max(amax, a);
    c2 += a >= 2;
    c4 += a >= 4;
    c8 += a >= 8;
    c16 += a >= 16;
    sp += par[i];
    sp2 += (double)par[i] * par[i];
    const int x = i % B, y = i / B;
    if (x + 1 < B) {
      const double d = std::abs(par[i + 1] - par[i]);
      gx += d;
      gmax = std::max(gmax, d);
    }
    if (y + 1 < B) {
      const double d = std::abs(par[i + B] - par[i]);
      gy += d;
      gmax = std::max(gmax, d);
    }
  }
  const double mean = sa / S, var = std::max(0.0, sa2 / S - mean * mean);
  const double pm = sp / S, pvar = std::max(0.0, sp2 / S - pm * pm);
  const double ng = (double)B * (B - 1);
  f[0] = (float)(level / 4.0);
  f[1] = ch == 0 ? 1.0f : 0.0f;
  f[2] = (float)(std::log2(1.0 + mean) / 8.0);
  f[3] = (float)(std::log2(1.0 + amax) / 8.0);
  f[4] = (float)(std::log2(1.0 + var) / 16.0);
  f[5] = (float)(c2 / S);
  f[6] = (float)(c4 / S);
  f[7] = (float)(c8 / S);
  f[8] = (float)(c16 / S);
  f[9] = (float)(std::log2(1.0 + gx / ng) / 8.0);
  f[10] = (float)(std::log2(1.0 + gy / ng) / 8.0);
  f[11] = (float)(std::log2(1.0 + gmax) / 8.0);
  f[12] = (float)(std::log2(1.0 + pvar) / 16.0);
  f[13] = (float)(q / 4.0);
  f[14] = (float)(std::log2(1.0 + (double)lambda_q16 / 65536.0) / 24.0);
  f[15] = (float)(B / 8.0);
}

int64_t control_rows(const Geometry &g) {
  int64_t rows = 0;
  for (int l = 0; l < g.L - 1; l++) rows += (int64_t)g.lu[l] * g.lv[l] * g.nb * 3;
  return rows;
}

static lfc_status encode_impl(const uint8_t *rgb, const lfc_params &p, std::vector<uint8_t> *out,
                              lfc_encode_stats *stats, lfc_control *ctl) {
  Geometry g;
  std::string why;
  if (make_geometry(p, g, &why) != LFC_OK) return fail(LFC_E_INVALID, "lfc_encode: " + why);
  const uint32_t mask = p.range_mask ? p.range_mask : kAllCodes;
  const int B = g.B, S = g.S, L = g.L, q = g.q, nv = g.nv();
  const int64_t plane = (int64_t)g.hp * g.wp, img = 3 * plane;

  // Level 0: padded YCoCg-R planes [nv][3][hp][wp] (Sec. 4), edge replication.
  std::vector<std::vector<int16_t>> lvl(L);
  lvl[0].resize((size_t)nv * img);
  parallel_for((int64_t)nv * g.hp, 64, [&](int64_t a, int64_t e) {
    for (int64_t r = a; r < e; r++) {
      const int vi = (int)(r / g.hp), y = (int)(r % g.hp);
      const int sy = std::min(y, g.H - 1);
      int16_t *dst = &lvl[0][(size_t)vi * img + (size_t)y * g.wp];
      for (int x = 0; x < g.wp; x++) {
        const uint8_t *px = rgb + (((size_t)vi * g.H + sy) * g.W + std::min(x, g.W - 1)) * 3;
        const int co = px[0] - px[2];
        const int t = px[2] + (co >> 1);
        const int cg = px[1] - t;
        dst[x] = (int16_t)(t + (cg >> 1));
        dst[x + plane] = (int16_t)co;
        dst[x + 2 * plane] = (int16_t)cg;
      }
    }
  });

  // Stage I: RKV^l = cluster mean of level l-1 with binomial weights (eqs. 1-2),
  // rounded to nearest (half up) over the members that exist.
  for (int l = 1; l < L; l++) {
    const int c = g.c[l], nodes = g.lu[l] * g.lv[l];
    int64_t pascal[9] = {1};
    for (int i = 1; i < c; i++)
      for (int k = i; k >= 1; k--) pascal[k] += pascal[k - 1];
    lvl[l].resize((size_t)nodes * img);
    parallel_for((int64_t)nodes * 3 * g.hp, 16, [&](int64_t a, int64_t e) {
      for (int64_t r = a; r < e; r++) {
        const int node = (int)(r / (3 * g.hp)), ch = (int)(r / g.hp % 3), y = (int)(r % g.hp);
        const int nx = node % g.lu[l], ny = node / g.lu[l];
        const int16_t *src[64];
        int64_t wgt[64];
        int cnt = 0;
        int64_t wsum = 0;
        for (int yy = ny * c; yy < std::min(ny * c + c, g.lv[l - 1]); yy++)
          for (int xx = nx * c; xx < std::min(nx * c + c, g.lu[l - 1]); xx++) {
            src[cnt] = &lvl[l - 1][(size_t)(yy * g.lu[l - 1] + xx) * img + (size_t)ch * plane + (size_t)y * g.wp];
            wgt[cnt] = pascal[xx - nx * c] * pascal[yy - ny * c];
            wsum += wgt[cnt++];
          }
        int16_t *dst = &lvl[l][(size_t)node * img + (size_t)ch * plane + (size_t)y * g.wp];
        for (int x = 0; x < g.wp; x++) {
          int64_t acc = wsum / 2;
          for (int k = 0; k < cnt; k++) acc += wgt[k] * src[k][x];
          dst[x] = (int16_t)floor_div(acc, wsum);
        }
      }
    });
  }

  TreeTables tt;
  build_tree_tables(g, tt);

  // allowed ranges by increasing size; a block takes the first that holds its values
  std::vector<std::pair<int, int>> ranges;
  for (int k = 0; k < kNumCodes; k++)
    if ((mask >> k) & 1u) ranges.push_back({range_code(k).bound, k});
  std::sort(ranges.begin(), ranges.end());

  // Stage II: closed-loop residual tree, top down (eq. 3 and the re-computed
  // RKVs of Sec. 3.2).  code_tab[g*n_srv + s] = range code or -1,
  // zv[(g*n_srv + s)*S + i] = zigzagged quantised residuals.
  const size_t nsg = (size_t)g.ng * g.n_srv;
  std::vector<int8_t> code_tab(std::max<size_t>(nsg, 1), -1);
  std::vector<uint16_t> zv(std::max<size_t>(nsg * S, 1), 0);
  std::vector<std::vector<int16_t>> rec(L);
  std::atomic<int> err{0};
  const int mode = ctl ? ctl->mode : LFC_CTL_GLOBAL;
  const int64_t lam = ctl ? ctl->lambda_q16 : 0;
  std::atomic<int64_t> fallbacks{0};
  std::vector<float> feat, pconf;
  std::vector<int8_t> pcls, prng;
  int64_t rowbase = 0;   // control row of the level's first (node, block, channel)
  for (int l = L - 2; l >= 0 && !err.load(); l--) {
    const int nodes = g.lu[l] * g.lv[l], cp = g.c[l + 1];
    rec[l].resize((size_t)nodes * img);
    const std::vector<int16_t> &prec = (l + 1 == L - 1) ? lvl[L - 1] : rec[l + 1];
    // one block of one channel: own samples, parent reconstruction, residuals
    auto load = [&](int64_t pair, int ch, int32_t *own, int32_t *par, int32_t *v) {
      const int node = (int)(pair / g.nb), b = (int)(pair % g.nb);
      const int nx = node % g.lu[l], ny = node / g.lu[l];
      const int parent = (ny / cp) * g.lu[l + 1] + nx / cp;
      const int bx = b % g.nbx, by = b / g.nbx;
      const size_t base = (size_t)ch * plane + (size_t)by * B * g.wp + (size_t)bx * B;
      const int16_t *po = &lvl[l][(size_t)node * img + base];
      const int16_t *pp = &prec[(size_t)parent * img + base];
      for (int i = 0; i < S; i++) {
        const size_t d = (size_t)(i / B) * g.wp + i % B;
        own[i] = po[d];
        par[i] = pp[d];
        v[i] = own[i] - par[i];
      }
    };
    const int64_t pairs = (int64_t)nodes * g.nb;
    const int64_t chunk = mode == LFC_CTL_MLP ? std::min<int64_t>(pairs, (int64_t)1 << 19) : pairs;
    for (int64_t c0 = 0; c0 < pairs && !err.load(); c0 += chunk) {
      const int64_t c1 = std::min(pairs, c0 + chunk);
      if (mode == LFC_CTL_MLP) {
        // features of the chunk, then the network's classes on the GPU
        const int64_t nr = (c1 - c0) * 3;
        feat.resize((size_t)nr * LFC_CTL_FEATURES);
        pcls.resize((size_t)nr);
        prng.resize((size_t)nr);
        pconf.resize((size_t)nr);
        parallel_for(c1 - c0, 256, [&](int64_t a, int64_t e) {
          int32_t own[64], par[64], v[64];
          for (int64_t r = a; r < e; r++)
            for (int ch = 0; ch < 3; ch++) {
              load(c0 + r, ch, own, par, v);
              block_features(v, par, B, l, ch, q, lam, &feat[(size_t)(r * 3 + ch) * LFC_CTL_FEATURES]);
            }
        });
        if (lfc_status st = mlp_infer_rows(ctl->d_mlp, feat.data(), nr, pcls.data(), prng.data(), pconf.data(),
                                           ctl->stream))
          return st;
      }
      parallel_for(c1 - c0, 256, [&](int64_t a, int64_t e) {
        int32_t own[64], par[64], v[64];
        Candidate cd, cs;
        for (int64_t r = a; r < e && !err.load(std::memory_order_relaxed); r++) {
          const int64_t pair = c0 + r;
          const int node = (int)(pair / g.nb), b = (int)(pair % g.nb);
          const int sidx = tt.serial[l][node];
          const int bx = b % g.nbx, by = b / g.nbx;
          for (int ch = 0; ch < 3; ch++) {
            load(pair, ch, own, par, v);
            const int64_t row = rowbase + pair * 3 + ch;
            if (mode == LFC_CTL_GLOBAL) {
              // the paper's global thresholds: pixel level, then block energy
              int64_t energy = 0;
              for (int i = 0; i < S; i++) {
                if (std::abs(v[i]) < p.pix_threshold) v[i] = 0;
                energy += std::abs(v[i]);
              }
              bool keep = energy > p.blk_threshold;
              uint32_t zmax = 0;
              if (keep) {
                bool nz = false;
                for (int i = 0; i < S; i++) {
                  v[i] = quantize_sample(v[i], q);
                  nz |= v[i] != 0;
                  zmax = std::max<uint32_t>(zmax, zz_encode(v[i]));
                }
                keep = nz;
              }
              cd.code = -1;
              if (keep) {
                for (const auto &rg : ranges)
                  if ((uint32_t)rg.first > zmax) {
                    cd.code = rg.second;
                    break;
                  }
                if (cd.code < 0) {
                  err.store(1);
                  return;
                }
              }
              for (int i = 0; i < S; i++) cd.qv[i] = keep ? v[i] : 0;
            } else {
              const bool need_search = mode == LFC_CTL_SEARCH || ctl->search_classes || ctl->search_ranges;
              int sc = -1;
              if (need_search) {
                sc = search_class(v, own, par, S, q, ch, lam, ranges, cs);
                if (ctl->search_classes) ctl->search_classes[row] = (int8_t)sc;
                if (ctl->search_ranges) ctl->search_ranges[row] = (int8_t)(cs.code < 0 ? LFC_CTL_ABSENT : cs.code);
              }
              if (ctl->features && mode != LFC_CTL_MLP) block_features(v, par, B, l, ch, q, lam, ctl->features + row * LFC_CTL_FEATURES);
              int cls;
              if (mode == LFC_CTL_SEARCH) {
                cls = sc;
                cd = cs;
              } else {
                int rng;
                bool fallback = false;
                if (mode == LFC_CTL_TABLE) {
                  cls = ctl->classes[row];
                  rng = ctl->ranges[row];
                  if (cls < 0 || cls >= LFC_CTL_CLASSES || rng < 0 || rng > LFC_CTL_ABSENT ||
                      (rng < LFC_CTL_ABSENT && !((mask >> rng) & 1u))) {
                    err.store(3);
                    return;
                  }
                } else {
                  const size_t pr = (size_t)((pair - c0) * 3 + ch);
                  if (ctl->features)
                    std::memcpy(ctl->features + row * LFC_CTL_FEATURES, &feat[pr * LFC_CTL_FEATURES],
                                sizeof(float) * LFC_CTL_FEATURES);
                  cls = pcls[pr];
                  rng = prng[pr];
                  fallback = !(pconf[pr] >= ctl->min_confidence);
                  if (!fallback && rng < LFC_CTL_ABSENT && !((mask >> rng) & 1u)) {
                    // a range the stream may not use: the values' own range
                    apply_class(v, own, par, S, q, cls, -1, ranges, cd);
                    rng = cd.code < 0 ? LFC_CTL_ABSENT : cd.code;
                  }
                }
                if (!fallback) {
                  apply_class(v, own, par, S, q, cls, rng, ranges, cd);
                  if (!cd.ok) {
                    if (mode == LFC_CTL_TABLE) {
                      err.store(2);
                      return;
                    }
                    fallback = true;
                  }
                }
                if (fallback) {
                  if (sc < 0) sc = search_class(v, own, par, S, q, ch, lam, ranges, cs);
                  cls = sc;
                  cd = cs;
                  fallbacks.fetch_add(1, std::memory_order_relaxed);
                }
              }
              if (ctl->classes && mode != LFC_CTL_TABLE) ctl->classes[row] = (int8_t)cls;
              if (ctl->ranges && mode != LFC_CTL_TABLE) ctl->ranges[row] = (int8_t)(cd.code < 0 ? LFC_CTL_ABSENT : cd.code);
            }
            const bool keep = cd.code >= 0;
            if (keep) {
              const size_t key = (size_t)(3 * b + ch) * g.n_srv + sidx;
              code_tab[key] = (int8_t)cd.code;
              for (int i = 0; i < S; i++) zv[key * S + i] = zz_encode(cd.qv[i]);
            }
            int16_t *dst = &rec[l][(size_t)node * img + (size_t)ch * plane + (size_t)by * B * g.wp + (size_t)bx * B];
            for (int i = 0; i < S; i++) {
              const int32_t x = par[i] + (keep ? cd.qv[i] * (1 << q) : 0);
              if (x < -32768 || x > 32767) {
                err.store(2);
                return;
              }
              dst[(size_t)(i / B) * g.wp + i % B] = (int16_t)x;
            }
          }
        }
      });
    }
    rowbase += pairs * 3;
    if (err.load()) break;
    if (l + 1 < L - 1) std::vector<int16_t>().swap(rec[l + 1]);  // no longer needed
  }
  if (ctl) ctl->fallbacks = fallbacks.load();
  if (err.load() == 1) return fail(LFC_E_RANGE, "lfc_encode: a residual block needs a BISE range the mask does not allow");
  if (err.load() == 2) return fail(LFC_E_RANGE, "lfc_encode: a reconstructed sample leaves int16");
  if (err.load() == 3) return fail(LFC_E_INVALID, "lfc_encode_ctl: a class table entry is out of range or names a range the mask excludes");
  if (stats) {
    // eq. 5 per view and channel on the unpadded area, eq. 4, mean over views
    const std::vector<int16_t> &r0 = L > 1 ? rec[0] : lvl[0];
    std::vector<double> sse((size_t)nv * 3);
    parallel_for(nv * 3, 1, [&](int64_t a, int64_t e) {
      for (int64_t r = a; r < e; r++) {
        const size_t o = (size_t)r * plane;
        double se = 0;
        for (int y = 0; y < g.H; y++)
          for (int x = 0; x < g.W; x++) {
            const double d = (double)r0[o + (size_t)y * g.wp + x] - (double)lvl[0][o + (size_t)y * g.wp + x];
            se += d * d;
          }
        sse[r] = se;
      }
    });
    encode_stats_from_sse(sse, nv, g.W, g.H, stats);
    std::fill(stats->code_hist, stats->code_hist + kNumCodes, 0);
    stats->present_blocks = 0;
    for (size_t i = 0; i < nsg; i++)
      if (code_tab[i] >= 0) {
        stats->code_hist[code_tab[i]]++;
        stats->present_blocks++;
      }
  }
  for (int l = 0; l < L - 1; l++) std::vector<int16_t>().swap(lvl[l]);
  rec.clear();

  // Stage III: location-gathered SRV stream (Sec. 3.4, Alg. 1).  Group
  // g = 3*b + c holds, for every node with a stored block at location b,
  // channel c: a bitmap of the nodes, their 5-bit range codes, then their
  // BISE payloads, in serial order.  An empty group stores nothing.
  std::vector<uint64_t> gwords(g.ng + 1, 0);
  parallel_for(g.ng, 64, [&](int64_t a, int64_t e) {
    for (int64_t gi = a; gi < e; gi++) {
      uint64_t present = 0, bits = 0;
      const int8_t *ct = &code_tab[(size_t)gi * g.n_srv];
      for (int s = 0; s < g.n_srv; s++)
        if (ct[s] >= 0) {
          present++;
          bits += bise_block_bits(ct[s], S);
        }
      gwords[gi] = present ? g.nbw + (5 * present + 31) / 32 + (bits + 31) / 32 : 0;
    }
  });
  std::vector<uint32_t> offsets(g.ng + 1);
  uint64_t acc = 0;
  for (int gi = 0; gi < g.ng; gi++) {
    offsets[gi] = (uint32_t)acc;
    acc += gwords[gi];
    if (acc > 0xFFFFFFF0ull) return fail(LFC_E_RANGE, "lfc_encode: stream exceeds 2^32 words");
  }
  offsets[g.ng] = (uint32_t)acc;
  const uint64_t srv_words = acc + 2;
  const uint64_t rkv_bytes = (uint64_t)g.n_top * g.nb * 3 * S * 2;
  const uint64_t rkv_off = kHeaderBytes, off_off = rkv_off + rkv_bytes;
  const uint64_t srv_off = off_off + 4ull * (g.ng + 1);
  if (stats) stats->stream_bytes = srv_off + 4 * srv_words;
  if (!out) return LFC_OK;
  try {
    out->assign(srv_off + 4 * srv_words, 0);
  } catch (const std::bad_alloc &) {
    return fail(LFC_E_NOMEM, "lfc_encode: out of host memory");
  }
  put_stream_header(out->data(), g, p, mask, rkv_off, off_off, srv_off);
  // RKVStream: the top level, stored raw as int16 [n_top][nb][3][B*B]
  {
    int16_t *dst = reinterpret_cast<int16_t *>(out->data() + rkv_off);
    const std::vector<int16_t> &top = lvl[L - 1];
    parallel_for((int64_t)g.n_top * g.nb, 1024, [&](int64_t a, int64_t e) {
      for (int64_t r = a; r < e; r++) {
        const int n = (int)(r / g.nb), b = (int)(r % g.nb), bx = b % g.nbx, by = b / g.nbx;
        for (int ch = 0; ch < 3; ch++)
          for (int i = 0; i < S; i++)
            dst[(size_t)r * 3 * S + ch * S + i] =
                top[(size_t)n * img + (size_t)ch * plane + (size_t)(by * B + i / B) * g.wp + bx * B + i % B];
      }
    });
  }
  std::memcpy(out->data() + off_off, offsets.data(), 4ull * (g.ng + 1));
  uint32_t *srv = reinterpret_cast<uint32_t *>(out->data() + srv_off);
  parallel_for(g.ng, 64, [&](int64_t a, int64_t e) {
    for (int64_t gi = a; gi < e; gi++) {
      if (!gwords[gi]) continue;
      uint32_t *w = srv + offsets[gi];
      const int8_t *ct = &code_tab[(size_t)gi * g.n_srv];
      uint64_t present = 0;
      for (int s = 0; s < g.n_srv; s++)
        if (ct[s] >= 0) {
          w[s >> 5] |= 1u << (s & 31);
          present++;
        }
      uint64_t cpos = 32ull * g.nbw;
      uint64_t ppos = 32ull * (g.nbw + (5 * present + 31) / 32);
      for (int s = 0; s < g.n_srv; s++) {
        if (ct[s] < 0) continue;
        put_field(w, cpos, (uint32_t)ct[s]);
        cpos += 5;
        ppos = pack_block(w, ppos, &zv[((size_t)gi * g.n_srv + s) * S], S, ct[s]);
      }
    }
  });
  return LFC_OK;
}

// ---------------------------------------------------------------------------
// stream validation and the block directory
// ---------------------------------------------------------------------------

struct Parsed {
  lfc_params p{};
  Geometry g;
  const uint8_t *rkv = nullptr;
  size_t rkv_bytes = 0;
  std::vector<uint32_t> off, srv;       // aligned copies; srv ends with the 2 zero words
  std::vector<uint32_t> dbase, poff;    // directory (built on request)
  std::vector<uint32_t> pbase;          // [ng+1] index in poff of each group's first stored block
  std::vector<uint32_t> dir2;           // [nb][nbw][3] (bitmap word, dbase) pairs, the three channels together
  uint64_t present = 0;
};

static inline uint32_t read_bits(const std::vector<uint32_t> &w, uint64_t pos, int n) {
  const uint64_t i = pos >> 5;
  uint64_t x = w[i];
  if (i + 1 < w.size()) x |= (uint64_t)w[i + 1] << 32;
  return (uint32_t)(x >> (pos & 31)) & (n == 32 ? 0xFFFFFFFFu : ((1u << n) - 1u));
}

template <typename T>
static T rd(const uint8_t *p) {
  T v;
  std::memcpy(&v, p, sizeof v);
  return v;
}

static lfc_status parse_validate(const void *stream, size_t bytes, Parsed &ps, bool build_dir) {
  const uint8_t *s = static_cast<const uint8_t *>(stream);
  auto corrupt = [](const std::string &m) { return fail(LFC_E_CORRUPT, "stream: " + m); };
  if (bytes < (size_t)kHeaderBytes) return corrupt("shorter than the header");
  if (std::memcmp(s, "RLFC", 4) != 0) return corrupt("bad magic");
  if (rd<uint16_t>(s + 4) != 1 || rd<uint16_t>(s + 6) != kHeaderBytes) return corrupt("unsupported version");
  lfc_params &p = ps.p;
  p.grid_u = rd<int32_t>(s + 8);
  p.grid_v = rd<int32_t>(s + 12);
  p.width = rd<int32_t>(s + 16);
  p.height = rd<int32_t>(s + 20);
  p.block = rd<int32_t>(s + 32);
  p.levels = rd<int32_t>(s + 36);
  p.quant_bits = rd<int32_t>(s + 40);
  if (p.levels < 1 || p.levels > kMaxLevels) return corrupt("levels");
  for (int i = 0; i < kMaxLevels; i++) {
    p.cluster[i] = rd<int32_t>(s + 48 + 4 * i);
    if (i >= p.levels - 1 && p.cluster[i] != 0) return corrupt("unused cluster entries must be 0");
  }
  p.pix_threshold = rd<int32_t>(s + 72);
  p.blk_threshold = rd<int32_t>(s + 76);
  p.range_mask = rd<uint32_t>(s + 80);
  if (p.range_mask == 0) return corrupt("empty range mask");
  std::string why;
  if (make_geometry(p, ps.g, &why) != LFC_OK) return corrupt("parameters: " + why);
  const Geometry &g = ps.g;
  if (rd<int32_t>(s + 24) != g.wp || rd<int32_t>(s + 28) != g.hp || rd<int32_t>(s + 44) != 3)
    return corrupt("padded size or channel count");
  if (rd<int32_t>(s + 84) != g.n_srv || rd<int32_t>(s + 88) != g.n_top || rd<int32_t>(s + 92) != g.nb ||
      rd<int32_t>(s + 96) != g.ng || rd<uint32_t>(s + 100) != 0)
    return corrupt("derived sizes");
  const uint64_t rkv_off = rd<uint64_t>(s + 104), off_off = rd<uint64_t>(s + 112), srv_off = rd<uint64_t>(s + 120);
  ps.rkv_bytes = (size_t)g.n_top * g.nb * 3 * g.S * 2;
  if (rkv_off != (uint64_t)kHeaderBytes || off_off != rkv_off + ps.rkv_bytes ||
      srv_off != off_off + 4ull * (g.ng + 1))
    return corrupt("section offsets");
  if (bytes < srv_off + 8 || (bytes - srv_off) % 4) return corrupt("truncated");
  ps.rkv = s + rkv_off;
  const uint64_t srv_words = (bytes - srv_off) / 4;
  ps.off.resize(g.ng + 1);
  std::memcpy(ps.off.data(), s + off_off, 4ull * (g.ng + 1));
  if (ps.off[0] != 0) return corrupt("first offset");
  for (int gi = 0; gi < g.ng; gi++)
    if (ps.off[gi + 1] < ps.off[gi]) return corrupt(fmt("offsets decrease at group %d", gi));
  if ((uint64_t)ps.off[g.ng] + 2 != srv_words) return corrupt("SRV section length");
  ps.srv.resize(srv_words);
  std::memcpy(ps.srv.data(), s + srv_off, 4 * srv_words);
  if (ps.srv[srv_words - 1] || ps.srv[srv_words - 2]) return corrupt("tail words");

  // every group: bitmap, codes, payload length, padding and digit fields
  const int S = g.S;
  const uint32_t mask = p.range_mask;
  std::vector<uint32_t> count(g.ng, 0);
  std::atomic<int64_t> bad_group{-1};
  parallel_for(g.ng, 256, [&](int64_t a, int64_t e) {
    for (int64_t gi = a; gi < e; gi++) {
      const uint64_t o0 = ps.off[gi], len = ps.off[gi + 1] - o0;
      if (!len) continue;
      auto bad = [&] {
        int64_t cur = -1;
        bad_group.compare_exchange_strong(cur, gi);
      };
      if (g.nbw == 0 || len < (uint64_t)g.nbw || len > (1u << 22)) { bad(); continue; }
      const uint32_t *bm = &ps.srv[o0];
      uint64_t P = 0;
      for (int w = 0; w < g.nbw; w++) P += __builtin_popcount(bm[w]);
      if ((g.n_srv & 31) && (bm[g.nbw - 1] >> (g.n_srv & 31))) { bad(); continue; }
      const uint64_t ncw = (5 * P + 31) / 32;
      if (P == 0 || len < g.nbw + ncw) { bad(); continue; }
      const uint64_t base = 32 * o0, cbit = base + 32ull * g.nbw;
      uint64_t bits = 0;
      bool ok = true;
      for (uint64_t r = 0; r < P && ok; r++) {
        const uint32_t k = read_bits(ps.srv, cbit + 5 * r, 5);
        if (k >= (uint32_t)kNumCodes || !((mask >> k) & 1u)) ok = false;
        else bits += bise_block_bits((int)k, S);
      }
      if (!ok || len != g.nbw + ncw + (bits + 31) / 32) { bad(); continue; }
      // padding after the codes and after the payload must be zero
      for (uint64_t pos = cbit + 5 * P; pos < base + 32ull * (g.nbw + ncw) && ok; pos++)
        ok = !read_bits(ps.srv, pos, 1);
      for (uint64_t pos = base + 32ull * (g.nbw + ncw) + bits; pos < base + 32 * len && ok; pos++)
        ok = !read_bits(ps.srv, pos, 1);
      // digit fields below radix^k
      uint64_t pp = base + 32ull * (g.nbw + ncw);
      for (uint64_t r = 0; r < P && ok; r++) {
        const RangeCode rc = range_code((int)read_bits(ps.srv, cbit + 5 * r, 5));
        if (rc.kind) {
          const int glen = rc.kind == 1 ? 5 : 3, radix = rc.kind == 1 ? 3 : 5, full = rc.kind == 1 ? 8 : 7;
          uint64_t fp = pp;
          for (int i0 = 0; i0 < S && ok; i0 += glen) {
            const int k = std::min(glen, S - i0), wdt = (full * k + glen - 1) / glen;
            uint32_t lim = 1;
            for (int j = 0; j < k; j++) lim *= radix;
            ok = read_bits(ps.srv, fp, wdt) < lim;
            fp += wdt;
          }
        }
        pp += S * rc.m + digit_plane_bits(rc.kind, S);
      }
      if (!ok) { bad(); continue; }
      count[gi] = (uint32_t)P;
    }
  });
  if (bad_group.load() >= 0) return corrupt(fmt("group %lld is malformed", (long long)bad_group.load()));
  ps.present = 0;
  for (int gi = 0; gi < g.ng; gi++) ps.present += count[gi];
  if (!build_dir) return LFC_OK;
  if (ps.present > 0xFFFFFFF0ull) return fail(LFC_E_UNSUPPORTED, "more than 2^32 stored blocks");

  // Directory for random access (built once, as Sec. 3.5 locates blocks at
  // initialisation): dbase[g][w] = index in poff of the first stored node of
  // bitmap word w; poff[i] = (payload bit offset within the group << 5) | code.
  std::vector<uint32_t> &pbase = ps.pbase;
  pbase.assign(g.ng + 1, 0);
  for (int gi = 0; gi < g.ng; gi++) pbase[gi + 1] = pbase[gi] + count[gi];
  ps.dbase.assign((size_t)g.ng * g.nbw, 0);
  ps.poff.assign(std::max<uint64_t>(ps.present, 1), 0);
  parallel_for(g.ng, 256, [&](int64_t a, int64_t e) {
    for (int64_t gi = a; gi < e; gi++) {
      uint32_t idx = pbase[gi];
      const uint64_t o0 = ps.off[gi];
      const bool empty = ps.off[gi + 1] == o0;
      for (int w = 0; w < g.nbw; w++) {
        ps.dbase[(size_t)gi * g.nbw + w] = idx;
        if (!empty) idx += __builtin_popcount(ps.srv[o0 + w]);
      }
      if (empty) continue;
      const uint64_t P = count[gi], base = 32 * o0;
      const uint64_t cbit = base + 32ull * g.nbw;
      uint64_t rel = 32ull * (g.nbw + (5 * P + 31) / 32);
      for (uint64_t r = 0; r < P; r++) {
        const uint32_t k = read_bits(ps.srv, cbit + 5 * r, 5);
        ps.poff[pbase[gi] + r] = (uint32_t)(rel << 5) | k;
        rel += bise_block_bits((int)k, S);
      }
    }
  });
  // the same lookups laid out for random access: for block b and bitmap word
  // w, the three channels' (bitmap word, directory index) pairs side by side,
  // so one access reads them from one cache line instead of four
  ps.dir2.assign((size_t)g.nb * g.nbw * 3 * 2, 0);
  parallel_for(g.nb, 1024, [&](int64_t a, int64_t e) {
    for (int64_t b = a; b < e; b++)
      for (int w = 0; w < g.nbw; w++)
        for (int c = 0; c < 3; c++) {
          const size_t gi = 3 * (size_t)b + c, at = (((size_t)b * g.nbw + w) * 3 + c) * 2;
          ps.dir2[at] = ps.off[gi + 1] == ps.off[gi] ? 0u : ps.srv[ps.off[gi] + w];
          ps.dir2[at + 1] = ps.dbase[gi * g.nbw + w];
        }
  });
  return LFC_OK;
}

}  // namespace lfc

// ---------------------------------------------------------------------------
// exported calls
// ---------------------------------------------------------------------------

using namespace lfc;

extern "C" const char *lfc_last_error(void) { return g_last_error.c_str(); }

extern "C" lfc_status lfc_encode_ex(const uint8_t *rgb, const lfc_params *p, void **stream_out, size_t *bytes_out,
                                    lfc_encode_stats *stats) {
  if (!rgb || !p || (!stream_out) != (!bytes_out)) return fail(LFC_E_INVALID, "lfc_encode: null argument");
  if (stream_out) {
    *stream_out = nullptr;
    *bytes_out = 0;
  }
  std::vector<uint8_t> buf;
  lfc_status st;
  try {
    st = encode_impl(rgb, *p, stream_out ? &buf : nullptr, stats, nullptr);
  } catch (const std::bad_alloc &) {
    return fail(LFC_E_NOMEM, "lfc_encode: out of host memory");
  }
  if (st != LFC_OK || !stream_out) return st;
  void *mem = std::malloc(buf.size());
  if (!mem) return fail(LFC_E_NOMEM, "lfc_encode: out of host memory");
  std::memcpy(mem, buf.data(), buf.size());
  *stream_out = mem;
  *bytes_out = buf.size();
  return LFC_OK;
}

extern "C" int64_t lfc_control_rows(const lfc_params *p) {
  if (!p) return -1;
  Geometry g;
  if (make_geometry(*p, g, nullptr) != LFC_OK) return -1;
  return control_rows(g);
}

extern "C" lfc_status lfc_encode_ctl(const uint8_t *rgb, const lfc_params *p, lfc_control *ctl, void **stream_out,
                                     size_t *bytes_out, lfc_encode_stats *stats) {
  if (!rgb || !p || !ctl || (!stream_out) != (!bytes_out)) return fail(LFC_E_INVALID, "lfc_encode_ctl: null argument");
  if (stream_out) {
    *stream_out = nullptr;
    *bytes_out = 0;
  }
  const int m = ctl->mode;
  if (m != LFC_CTL_GLOBAL && m != LFC_CTL_SEARCH && m != LFC_CTL_TABLE && m != LFC_CTL_MLP)
    return fail(LFC_E_INVALID, "lfc_encode_ctl: unknown mode");
  if (ctl->lambda_q16 < 0 || ctl->lambda_q16 > ((int64_t)1 << 52))
    return fail(LFC_E_INVALID, "lfc_encode_ctl: lambda_q16 must be 0..2^52");
  Geometry g;
  std::string why;
  if (make_geometry(*p, g, &why) != LFC_OK) return fail(LFC_E_INVALID, "lfc_encode_ctl: " + why);
  const bool tables = ctl->classes || ctl->ranges || ctl->features || ctl->search_classes || ctl->search_ranges;
  if (tables && ctl->rows != control_rows(g))
    return fail(LFC_E_INVALID, "lfc_encode_ctl: rows must equal lfc_control_rows(p)");
  if (m == LFC_CTL_TABLE && (!ctl->classes || !ctl->ranges))
    return fail(LFC_E_INVALID, "lfc_encode_ctl: TABLE mode needs classes and ranges");
  if (m == LFC_CTL_MLP && !ctl->d_mlp) return fail(LFC_E_INVALID, "lfc_encode_ctl: MLP mode needs device weights");
  if (m == LFC_CTL_GLOBAL && tables)
    return fail(LFC_E_INVALID, "lfc_encode_ctl: the GLOBAL mode fills no tables");
  ctl->fallbacks = 0;
  std::vector<uint8_t> buf;
  lfc_status st;
  try {
    st = encode_impl(rgb, *p, stream_out ? &buf : nullptr, stats, ctl);
  } catch (const std::bad_alloc &) {
    return fail(LFC_E_NOMEM, "lfc_encode_ctl: out of host memory");
  }
  if (st != LFC_OK || !stream_out) return st;
  void *mem = std::malloc(buf.size());
  if (!mem) return fail(LFC_E_NOMEM, "lfc_encode_ctl: out of host memory");
  std::memcpy(mem, buf.data(), buf.size());
  *stream_out = mem;
  *bytes_out = buf.size();
  return LFC_OK;
}

extern "C" lfc_status lfc_encode(const uint8_t *rgb, const lfc_params *p, void **stream_out, size_t *bytes_out) {
  if (!stream_out || !bytes_out) return fail(LFC_E_INVALID, "lfc_encode: null argument");
  return lfc_encode_ex(rgb, p, stream_out, bytes_out, nullptr);
}

extern "C" void lfc_free(void *ptr) { std::free(ptr); }

extern "C" lfc_status lfc_validate(const void *stream, size_t bytes, lfc_params *p_out) {
  if (!stream) return fail(LFC_E_INVALID, "lfc_validate: null stream");
  Parsed ps;
  lfc_status st;
  try {
    st = parse_validate(stream, bytes, ps, false);
  } catch (const std::bad_alloc &) {
    return fail(LFC_E_NOMEM, "lfc_validate: out of host memory");
  }
  if (st == LFC_OK && p_out) *p_out = ps.p;
  return st;
}

static size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

extern "C" lfc_status lfc_open(const void *stream, size_t bytes, hipStream_t s, lfc_lf **out) {
  return lfc_open_ex(stream, bytes, nullptr, s, out);
}

extern "C" lfc_status lfc_open_ex(const void *stream, size_t bytes, const lfc_open_config *cfg, hipStream_t s,
                                  lfc_lf **out) {
  if (!stream || !out) return fail(LFC_E_INVALID, "lfc_open: null argument");
  *out = nullptr;
  Parsed ps;
  TreeTables tt;
  try {
    lfc_status st = parse_validate(stream, bytes, ps, true);
    if (st != LFC_OK) return st;
    build_tree_tables(ps.g, tt);
  } catch (const std::bad_alloc &) {
    return fail(LFC_E_NOMEM, "lfc_open: out of host memory");
  }
  const Geometry &g = ps.g;
  // sections of the single device allocation
  struct Part {
    const void *src;
    size_t bytes;
    size_t at;
  };
  static const uint32_t zeros[64] = {0};
  // tile capacity of the whole-field kernel (the caller's, else the default;
  // lfc_tune_decode measures the choice): at least one run of kBatch leaves
  // with four ancestors, 8 nodes of 64/B blocks
  int tile_cap = tile_blocks(ps.g.B);
  if (cfg && cfg->tile_blocks) {
    if (cfg->tile_blocks < 512 / ps.g.B || cfg->tile_blocks > 2048 || cfg->tile_blocks % 8)
      return fail(LFC_E_INVALID, "lfc_open: tile_blocks must be a multiple of 8 in 512/B..2048 (or 0)");
    tile_cap = cfg->tile_blocks;
  }
  StripTables stt;
  try {
    make_strip_tables(ps.g, ps.off, ps.srv, ps.dbase, ps.poff, tt.batch, tile_cap, stt);
  } catch (const std::bad_alloc &) {
    return fail(LFC_E_NOMEM, "lfc_open: out of host memory");
  }
  const std::vector<uint32_t> &sched = stt.sched, &strip_off = stt.strip_off, &order = stt.order;
  // the colour kernel's strip tables (tile of the default capacity, which
  // holds a run of kBatch leaves and four ancestors in all three channels)
  const int tile_cap_rgb = tile_blocks(ps.g.B);
  StripTables rgbt;
  try {
    make_strip_tables_rgb(ps.g, ps.off, ps.srv, ps.dbase, ps.poff, tt.batch, tile_cap_rgb, rgbt);
  } catch (const std::bad_alloc &) {
    return fail(LFC_E_NOMEM, "lfc_open: out of host memory");
  }
  Part parts[17] = {
      {ps.rkv, ps.rkv_bytes, 0},
      {ps.off.data(), ps.off.size() * 4, 0},
      {ps.srv.data(), ps.srv.size() * 4, 0},
      {ps.dbase.data(), ps.dbase.size() * 4, 0},
      {ps.poff.data(), ps.poff.size() * 4, 0},
      {tt.path.data(), tt.path.size() * 4, 0},
      {tt.root.data(), tt.root.size() * 4, 0},
      {tt.batch.data(), tt.batch.size() * 4, 0},
      {zeros, 4, 0},
      {ps.pbase.data(), ps.pbase.size() * 4, 0},
      {sched.data(), sched.size() * 4, 0},
      {strip_off.data(), strip_off.size() * 4, 0},
      {order.data(), order.size() * 4, 0},
      {rgbt.sched.data(), rgbt.sched.size() * 4, 0},
      {rgbt.strip_off.data(), rgbt.strip_off.size() * 4, 0},
      {rgbt.order.data(), rgbt.order.size() * 4, 0},
      {ps.dir2.data(), ps.dir2.size() * 4, 0},
  };
  size_t total = 0;
  for (auto &pt : parts) {
    pt.at = total;
    // the SRV section gets 64 spare zero words so wide bit-window reads stay inside
    total += align256(pt.bytes + (&pt == &parts[2] ? 256 : 0));
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(LFC_E_HIP, "lfc_open: no current device");
  void *base = nullptr;
  hipError_t he = hipMalloc(&base, total);
  if (he != hipSuccess) return fail(he == hipErrorOutOfMemory ? LFC_E_NOMEM : LFC_E_HIP,
                                    std::string("lfc_open: hipMalloc: ") + hipGetErrorString(he));
  char *d = static_cast<char *>(base);
  for (auto &pt : parts) {
    if (pt.bytes) he = hipMemcpyAsync(d + pt.at, pt.src, pt.bytes, hipMemcpyHostToDevice, s);
    if (he == hipSuccess && &pt == &parts[2])
      he = hipMemcpyAsync(d + pt.at + pt.bytes, zeros, 256, hipMemcpyHostToDevice, s);
    if (he != hipSuccess) break;
  }
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  if (he != hipSuccess) {
    (void)hipStreamSynchronize(s);
    (void)hipFree(base);
    return fail(LFC_E_HIP, std::string("lfc_open: copy to device: ") + hipGetErrorString(he));
  }
  lfc_lf *lf = new (std::nothrow) lfc_lf;
  if (!lf) {
    (void)hipFree(base);
    return fail(LFC_E_NOMEM, "lfc_open: out of host memory");
  }
  lf->params = ps.p;
  lf->geo = g;
  lf->tile_cap = tile_cap;
  lf->device = dev;
  lf->stream_bytes = bytes;
  lf->present = ps.present;
  lf->d_base = base;
  lf->d_bytes = total;
  lf->d_rkv = reinterpret_cast<const int16_t *>(d + parts[0].at);
  lf->d_off = reinterpret_cast<const uint32_t *>(d + parts[1].at);
  lf->d_srv = reinterpret_cast<const uint32_t *>(d + parts[2].at);
  lf->d_dbase = reinterpret_cast<const uint32_t *>(d + parts[3].at);
  lf->d_poff = reinterpret_cast<const uint32_t *>(d + parts[4].at);
  lf->d_path = reinterpret_cast<const int32_t *>(d + parts[5].at);
  lf->d_root = reinterpret_cast<const int32_t *>(d + parts[6].at);
  lf->d_batch = reinterpret_cast<const int32_t *>(d + parts[7].at);
  lf->n_batch = (int)(tt.batch.size() / kBatchWords);
  lf->d_pbase = reinterpret_cast<const uint32_t *>(d + parts[9].at);
  lf->d_sched = reinterpret_cast<const uint32_t *>(d + parts[10].at);
  lf->d_strip_off = reinterpret_cast<const uint32_t *>(d + parts[11].at);
  lf->d_order = reinterpret_cast<const uint32_t *>(d + parts[12].at);
  lf->d_sched_rgb = reinterpret_cast<const uint32_t *>(d + parts[13].at);
  lf->d_strip_off_rgb = reinterpret_cast<const uint32_t *>(d + parts[14].at);
  lf->d_order_rgb = reinterpret_cast<const uint32_t *>(d + parts[15].at);
  lf->d_dir2 = reinterpret_cast<const uint32_t *>(d + parts[16].at);
  lf->tile_cap_rgb = tile_cap_rgb;
  for (size_t st = 0; st + 1 < rgbt.strip_off.size(); st++)
    lf->rgb_max_chunks = std::max<int>(lf->rgb_max_chunks, (int)rgbt.sched[rgbt.strip_off[st]]);
  lf->d_err = reinterpret_cast<int32_t *>(d + parts[8].at);
  // LDS staging of the whole-field kernel is sized by the largest strip:
  // group words plus the strip's decode schedule
  lf->max_strip_words = stt.max_words;
  lf->strip_need = std::move(stt.need);
  *out = lf;
  return LFC_OK;
}

extern "C" int64_t lfc_stage_needs(const lfc_lf *lf, uint32_t *need, int64_t n) {
  if (!lf) return fail(LFC_E_INVALID, "lfc_stage_needs: null handle");
  const int64_t strips = (int64_t)(lf->strip_need.size() / 2);
  if (need)
    for (int64_t i = 0; i < std::min(n, strips) * 2; i++) need[i] = lf->strip_need[(size_t)i];
  return strips;
}

extern "C" lfc_status lfc_info(const lfc_lf *lf, lfc_info_t *info) {
  if (!lf || !info) return fail(LFC_E_INVALID, "lfc_info: null argument");
  info->params = lf->params;
  info->padded_width = lf->geo.wp;
  info->padded_height = lf->geo.hp;
  info->n_blocks = lf->geo.nb;
  info->n_groups = lf->geo.ng;
  info->n_srv = lf->geo.n_srv;
  info->n_top = lf->geo.n_top;
  info->stream_bytes = lf->stream_bytes;
  info->device_bytes = lf->d_bytes;
  info->present_blocks = lf->present;
  return LFC_OK;
}

extern "C" lfc_status lfc_check(const lfc_lf *lf, hipStream_t s) {
  if (!lf) return fail(LFC_E_INVALID, "lfc_check: null handle");
  hipError_t he = hipStreamSynchronize(s);
  int32_t flag = 0;
  if (he == hipSuccess) he = hipMemcpy(&flag, lf->d_err, 4, hipMemcpyDeviceToHost);
  if (he != hipSuccess) return fail(LFC_E_HIP, std::string("lfc_check: ") + hipGetErrorString(he));
  if (flag) {
    const int32_t zero = 0;
    he = hipMemcpy(lf->d_err, &zero, 4, hipMemcpyHostToDevice);
    if (he != hipSuccess) return fail(LFC_E_HIP, std::string("lfc_check: ") + hipGetErrorString(he));
    return fail(LFC_E_INVALID, "a decode request named a view or block out of range");
  }
  return LFC_OK;
}

// Measured choice of the whole-field kernel's tile capacity: the strip
// tables are rebuilt on the host for each candidate (the directory and run
// table come back from the device) and the decode is timed with each.
extern "C" lfc_status lfc_tune_decode(lfc_lf *lf, int16_t *d_out, int32_t reps, lfc_decode_tuning *res,
                                      hipStream_t s) {
  if (!lf || !d_out || !res) return fail(LFC_E_INVALID, "lfc_tune_decode: null argument");
  if (reps < 1 || reps > 1000) return fail(LFC_E_INVALID, "lfc_tune_decode: reps must be 1..1000");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != lf->device)
    return fail(LFC_E_INVALID, "lfc_tune_decode: the light field was opened on another device");
  std::memset(res, 0, sizeof *res);
  const Geometry &g = lf->geo;
  const int nv = g.nv();
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return fail(LFC_E_HIP, "lfc_tune_decode: events");
  }
  // time the current tables with the handle's current staging
  auto timed = [&](float *ms) -> lfc_status {
    lfc_status st = lfc_decode_blocks(lf, nullptr, nv, LFC_LAYOUT_IMAGES, d_out, s);
    if (st != LFC_OK) return st;
    if (hipEventRecord(e0, s) != hipSuccess) return fail(LFC_E_HIP, "lfc_tune_decode: event record");
    for (int r = 0; r < reps && st == LFC_OK; r++) st = lfc_decode_blocks(lf, nullptr, nv, LFC_LAYOUT_IMAGES, d_out, s);
    if (st != LFC_OK) return st;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(ms, e0, e1) != hipSuccess)
      return fail(LFC_E_HIP, "lfc_tune_decode: timing");
    *ms /= (float)reps;
    return LFC_OK;
  };
  struct Saved {
    int cap;
    const uint32_t *sched, *strip_off, *order;
    std::vector<uint32_t> need;
    uint32_t max_words;
    void *own;
  };
  auto save = [&]() {
    return Saved{lf->tile_cap, lf->d_sched, lf->d_strip_off, lf->d_order, lf->strip_need, lf->max_strip_words,
                 lf->d_sched_own};
  };
  auto restore = [&](const Saved &v) {
    lf->tile_cap = v.cap;
    lf->d_sched = v.sched;
    lf->d_strip_off = v.strip_off;
    lf->d_order = v.order;
    lf->strip_need = v.need;
    lf->max_strip_words = v.max_words;
    lf->d_sched_own = v.own;
  };
  std::vector<Saved> cands;
  std::vector<int> tried_cand;        // per result: the table set it was timed with
  const int64_t stage0 = lf->stage_cap;
  lfc_status st = LFC_OK;
  float ms = 0.0f;
  // the current table set with and without staging
  auto time_both = [&](int cand) -> lfc_status {
    for (int staged = 0; staged < 2 && res->n_tried < LFC_TUNE_DECODE_MAX; staged++) {
      lf->stage_cap = staged ? -1 : 0;
      const lfc_status ts = timed(&ms);
      if (ts != LFC_OK) return ts;
      const int k = res->n_tried++;
      res->tile_blocks[k] = lf->tile_cap;
      res->staged[k] = staged;
      res->ms[k] = ms;
      tried_cand.push_back(cand);
    }
    return LFC_OK;
  };
  cands.push_back(save());
  st = time_both(0);
  try {
    // host copies of what the strip tables are built from
    std::vector<uint32_t> off, srv, dbase, poff;
    std::vector<int32_t> batch((size_t)lf->n_batch * kBatchWords);
    off.resize((size_t)g.ng + 1);
    if (st == LFC_OK && hipMemcpy(off.data(), lf->d_off, 4 * off.size(), hipMemcpyDeviceToHost) != hipSuccess)
      st = fail(LFC_E_HIP, "lfc_tune_decode: copy of the offsets");
    if (st == LFC_OK) {
      srv.resize((size_t)off[g.ng] + 2);
      dbase.resize((size_t)g.ng * g.nbw);
      poff.resize(std::max<uint64_t>(lf->present, 1));
      if (hipMemcpy(srv.data(), lf->d_srv, 4 * srv.size(), hipMemcpyDeviceToHost) != hipSuccess ||
          hipMemcpy(dbase.data(), lf->d_dbase, 4 * dbase.size(), hipMemcpyDeviceToHost) != hipSuccess ||
          hipMemcpy(poff.data(), lf->d_poff, 4 * poff.size(), hipMemcpyDeviceToHost) != hipSuccess ||
          (!batch.empty() &&
           hipMemcpy(batch.data(), lf->d_batch, 4 * batch.size(), hipMemcpyDeviceToHost) != hipSuccess))
        st = fail(LFC_E_HIP, "lfc_tune_decode: copy of the directory");
    }
    const int c0 = tile_blocks(g.B);
    const int fr[4] = {3, 5, 6, 7};   // quarters of the default capacity besides 4/4
    for (int fi = 0; fi < 4 && st == LFC_OK && res->n_tried < LFC_TUNE_DECODE_MAX; fi++) {
      const int cap = std::min(2048, std::max(512 / g.B, c0 * fr[fi] / 4 / 8 * 8));
      bool seen = false;
      for (const Saved &v : cands) seen |= v.cap == cap;
      if (seen || g.L < 2) continue;
      StripTables t;
      make_strip_tables(g, off, srv, dbase, poff, batch, cap, t);
      const size_t a0 = 0, a1 = align256(4 * t.sched.size()), a2 = a1 + align256(4 * t.strip_off.size());
      const size_t total = a2 + align256(4 * t.order.size());
      void *buf = nullptr;
      if (hipMalloc(&buf, total) != hipSuccess) {
        (void)hipGetLastError();
        break;   // no room for another table set: keep what was measured
      }
      char *d = static_cast<char *>(buf);
      if (hipMemcpy(d + a0, t.sched.data(), 4 * t.sched.size(), hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(d + a1, t.strip_off.data(), 4 * t.strip_off.size(), hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(d + a2, t.order.data(), 4 * t.order.size(), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(buf);
        st = fail(LFC_E_HIP, "lfc_tune_decode: copy of the strip tables");
        break;
      }
      lf->tile_cap = cap;
      lf->d_sched = reinterpret_cast<const uint32_t *>(d + a0);
      lf->d_strip_off = reinterpret_cast<const uint32_t *>(d + a1);
      lf->d_order = reinterpret_cast<const uint32_t *>(d + a2);
      lf->strip_need = std::move(t.need);
      lf->max_strip_words = t.max_words;
      lf->d_sched_own = buf;
      cands.push_back(save());
      const int n_before = res->n_tried;
      lfc_status ts = time_both((int)cands.size() - 1);
      if (ts == LFC_E_UNSUPPORTED) {   // the tile does not fit the LDS: not a candidate
        (void)hipGetLastError();
        (void)hipFree(buf);
        cands.pop_back();
        res->n_tried = n_before;
        tried_cand.resize((size_t)n_before);
        restore(cands[0]);
        continue;
      }
      if (ts != LFC_OK) {
        st = ts;
        break;
      }
    }
  } catch (const std::bad_alloc &) {
    st = fail(LFC_E_NOMEM, "lfc_tune_decode: out of host memory");
  }
  (void)hipStreamSynchronize(s);
  if (st != LFC_OK || res->n_tried == 0) {
    // back to the tables and staging the handle had; free every set built here
    for (size_t k = 1; k < cands.size(); k++)
      if (cands[k].own) (void)hipFree(cands[k].own);
    restore(cands[0]);
    lf->stage_cap = stage0;
  } else {
    // keep the fastest; free the other table sets (and an earlier tuning's tables if replaced)
    int best = 0;
    for (int k = 1; k < res->n_tried; k++)
      if (res->ms[k] < res->ms[best]) best = k;
    res->best = best;
    const size_t keep = (size_t)tried_cand[(size_t)best];
    for (size_t k = 1; k < cands.size(); k++)
      if (k != keep && cands[k].own) (void)hipFree(cands[k].own);
    if (keep != 0 && cands[0].own) (void)hipFree(cands[0].own);
    restore(cands[keep]);
    lf->stage_cap = res->staged[best] ? -1 : 0;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

// Measured choice of the colour whole-field kernel's tile capacity, as
// lfc_tune_decode for the one-channel kernel: the colour strip tables are
// rebuilt for each candidate and lfc_decode_rgb of every view is timed.
extern "C" lfc_status lfc_tune_decode_rgb(lfc_lf *lf, uint32_t *d_out, int32_t reps, lfc_decode_tuning *res,
                                          hipStream_t s) {
  if (!lf || !d_out || !res) return fail(LFC_E_INVALID, "lfc_tune_decode_rgb: null argument");
  if (reps < 1 || reps > 1000) return fail(LFC_E_INVALID, "lfc_tune_decode_rgb: reps must be 1..1000");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != lf->device)
    return fail(LFC_E_INVALID, "lfc_tune_decode_rgb: the light field was opened on another device");
  std::memset(res, 0, sizeof *res);
  const Geometry &g = lf->geo;
  if (g.L < 2) return fail(LFC_E_UNSUPPORTED, "lfc_tune_decode_rgb: no residual levels to tile");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return fail(LFC_E_HIP, "lfc_tune_decode_rgb: events");
  }
  auto timed = [&](float *ms) -> lfc_status {
    lfc_status st = lfc_decode_rgb(lf, d_out, s);
    if (st != LFC_OK) return st;
    if (hipEventRecord(e0, s) != hipSuccess) return fail(LFC_E_HIP, "lfc_tune_decode_rgb: event record");
    for (int r = 0; r < reps && st == LFC_OK; r++) st = lfc_decode_rgb(lf, d_out, s);
    if (st != LFC_OK) return st;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(ms, e0, e1) != hipSuccess)
      return fail(LFC_E_HIP, "lfc_tune_decode_rgb: timing");
    *ms /= (float)reps;
    return LFC_OK;
  };
  struct Saved {
    int cap, max_chunks;
    const uint32_t *sched, *strip_off, *order;
    void *own;
  };
  auto save = [&]() {
    return Saved{lf->tile_cap_rgb, lf->rgb_max_chunks, lf->d_sched_rgb, lf->d_strip_off_rgb, lf->d_order_rgb,
                 lf->d_sched_rgb_own};
  };
  auto restore = [&](const Saved &v) {
    lf->tile_cap_rgb = v.cap;
    lf->rgb_max_chunks = v.max_chunks;
    lf->d_sched_rgb = v.sched;
    lf->d_strip_off_rgb = v.strip_off;
    lf->d_order_rgb = v.order;
    lf->d_sched_rgb_own = v.own;
  };
  std::vector<Saved> cands;
  cands.push_back(save());
  float ms = 0.0f;
  lfc_status st = timed(&ms);
  if (st == LFC_OK) {
    res->tile_blocks[0] = lf->tile_cap_rgb;
    res->ms[0] = ms;
    res->n_tried = 1;
  }
  try {
    std::vector<uint32_t> off, srv, dbase, poff;
    std::vector<int32_t> batch((size_t)lf->n_batch * kBatchWords);
    off.resize((size_t)g.ng + 1);
    if (st == LFC_OK && hipMemcpy(off.data(), lf->d_off, 4 * off.size(), hipMemcpyDeviceToHost) != hipSuccess)
      st = fail(LFC_E_HIP, "lfc_tune_decode_rgb: copy of the offsets");
    if (st == LFC_OK) {
      srv.resize((size_t)off[g.ng] + 2);
      dbase.resize((size_t)g.ng * g.nbw);
      poff.resize(std::max<uint64_t>(lf->present, 1));
      if (hipMemcpy(srv.data(), lf->d_srv, 4 * srv.size(), hipMemcpyDeviceToHost) != hipSuccess ||
          hipMemcpy(dbase.data(), lf->d_dbase, 4 * dbase.size(), hipMemcpyDeviceToHost) != hipSuccess ||
          hipMemcpy(poff.data(), lf->d_poff, 4 * poff.size(), hipMemcpyDeviceToHost) != hipSuccess ||
          (!batch.empty() &&
           hipMemcpy(batch.data(), lf->d_batch, 4 * batch.size(), hipMemcpyDeviceToHost) != hipSuccess))
        st = fail(LFC_E_HIP, "lfc_tune_decode_rgb: copy of the directory");
    }
    const int c0 = tile_blocks(g.B);
    const int fr[5] = {4, 5, 6, 7, 10};   // eighths of the default capacity besides 8/8
    for (int fi = 0; fi < 5 && st == LFC_OK && res->n_tried < LFC_TUNE_DECODE_MAX; fi++) {
      const int cap = std::min(2048, std::max(512 / g.B, c0 * fr[fi] / 8 / 8 * 8));
      bool seen = false;
      for (const Saved &v : cands) seen |= v.cap == cap;
      if (seen) continue;
      StripTables t;
      make_strip_tables_rgb(g, off, srv, dbase, poff, batch, cap, t);
      const size_t a1 = align256(4 * t.sched.size()), a2 = a1 + align256(4 * t.strip_off.size());
      const size_t total = a2 + align256(4 * t.order.size());
      void *buf = nullptr;
      if (hipMalloc(&buf, total) != hipSuccess) {
        (void)hipGetLastError();
        break;   // no room for another table set: keep what was measured
      }
      char *d = static_cast<char *>(buf);
      if (hipMemcpy(d, t.sched.data(), 4 * t.sched.size(), hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(d + a1, t.strip_off.data(), 4 * t.strip_off.size(), hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(d + a2, t.order.data(), 4 * t.order.size(), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(buf);
        st = fail(LFC_E_HIP, "lfc_tune_decode_rgb: copy of the strip tables");
        break;
      }
      int max_chunks = 1;
      for (size_t k = 0; k + 1 < t.strip_off.size(); k++)
        max_chunks = std::max<int>(max_chunks, (int)t.sched[t.strip_off[k]]);
      lf->tile_cap_rgb = cap;
      lf->rgb_max_chunks = max_chunks;
      lf->d_sched_rgb = reinterpret_cast<const uint32_t *>(d);
      lf->d_strip_off_rgb = reinterpret_cast<const uint32_t *>(d + a1);
      lf->d_order_rgb = reinterpret_cast<const uint32_t *>(d + a2);
      lf->d_sched_rgb_own = buf;
      cands.push_back(save());
      const lfc_status ts = timed(&ms);
      if (ts == LFC_E_UNSUPPORTED) {   // the tile does not fit the LDS: not a candidate
        (void)hipGetLastError();
        (void)hipFree(buf);
        cands.pop_back();
        restore(cands[0]);
        continue;
      }
      if (ts != LFC_OK) {
        st = ts;
        break;
      }
      res->tile_blocks[res->n_tried] = cap;
      res->ms[res->n_tried] = ms;
      res->n_tried++;
    }
  } catch (const std::bad_alloc &) {
    st = fail(LFC_E_NOMEM, "lfc_tune_decode_rgb: out of host memory");
  }
  (void)hipStreamSynchronize(s);
  if (st != LFC_OK || res->n_tried == 0) {
    for (size_t k = 1; k < cands.size(); k++)
      if (cands[k].own) (void)hipFree(cands[k].own);
    restore(cands[0]);
  } else {
    // the fastest, unless within 2 % of the capacity the handle had (run to
    // run noise is about that, and a move away should pay for itself)
    int best = 0;
    for (int k = 1; k < res->n_tried; k++)
      if (res->ms[k] < res->ms[best]) best = k;
    if (res->ms[best] > 0.98f * res->ms[0]) best = 0;
    res->best = best;
    // candidate k of the results is table set k (every timed set was kept)
    for (size_t k = 1; k < cands.size(); k++)
      if ((int)k != best && cands[k].own) (void)hipFree(cands[k].own);
    if (best != 0 && cands[0].own) (void)hipFree(cands[0].own);
    restore(cands[(size_t)best]);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

extern "C" lfc_status lfc_close(lfc_lf *lf) {
  if (!lf) return LFC_OK;
  if (lf->d_sched_own) (void)hipFree(lf->d_sched_own);
  if (lf->d_sched_rgb_own) (void)hipFree(lf->d_sched_rgb_own);
  hipError_t he = hipFree(lf->d_base);
  delete lf;
  if (he != hipSuccess) return fail(LFC_E_HIP, std::string("lfc_close: ") + hipGetErrorString(he));
  return LFC_OK;
}

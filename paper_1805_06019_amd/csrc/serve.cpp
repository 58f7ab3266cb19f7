// Batched rendering across light fields and the serving loop built on it.
//
// lfc_batch packs render requests into a table on the host, copies it to the
// device on the caller's stream and launches one multi-request render per
// block size.  lfc_server keeps a queue of requests, a device pool for their
// results and one engine thread that admits and launches batches on a few
// streams, polls their completion events and wakes the waiters.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.h"
#include "serve.h"

using lfc::fail;

namespace {

constexpr int kSlots = 4;       // request tables in flight per batch context
constexpr int kCtrStride = 16;  // words between two slots' counters (one cache line each)

// A request table: pinned host staging and its device copy.  `done` is
// recorded after the launches that read the table; the slot is rewritten
// only once it has fired, whatever stream the next call uses.
struct Slot {
  char *host = nullptr;     // pinned
  char *dev = nullptr;
  size_t cap = 0;           // bytes of each
  hipEvent_t done = nullptr;
  bool used = false;
};

// Decoded views of one light field (8-bit RGB words) for the colour path of
// a batch, kept by the context for later batches.  `done` is recorded after
// the launches that read it; a later batch, on any stream, waits for it
// before decoding into the same buffer.
struct Scratch {
  const lfc_lf *lf = nullptr;
  void *buf = nullptr;
  size_t bytes = 0;
  hipEvent_t done = nullptr;
  bool used = false;
};

}  // namespace

struct lfc_batch {
  int device = 0;
  Slot slot[kSlots];
  int next = 0;
  int32_t *d_err = nullptr;   // set by a batched decode that saw an out-of-range request
  uint32_t *d_ctr = nullptr;  // per slot, the persistent colour decode's two counters (zero between launches)
  std::deque<Scratch> scratch;   // (a deque: adding one keeps the others' addresses)
};

namespace {

void free_slot(Slot &sl) {
  if (sl.host) (void)hipHostFree(sl.host);
  if (sl.dev) (void)hipFree(sl.dev);
  sl.host = sl.dev = nullptr;
  sl.cap = 0;
}

lfc_status grow_slot(Slot &sl, size_t need) {
  if (need <= sl.cap) return LFC_OK;
  size_t cap = std::max<size_t>(need, 64 * lfc::render_req_bytes());
  cap = std::max(cap, sl.cap * 2);
  if (sl.used && hipEventSynchronize(sl.done) != hipSuccess) return fail(LFC_E_HIP, "lfc_batch_render: event wait");
  sl.used = false;
  free_slot(sl);
  if (hipHostMalloc(reinterpret_cast<void **>(&sl.host), cap, hipHostMallocDefault) != hipSuccess) {
    sl.host = nullptr;
    return fail(LFC_E_NOMEM, "lfc_batch_render: pinned staging");
  }
  if (hipMalloc(reinterpret_cast<void **>(&sl.dev), cap) != hipSuccess) {
    sl.dev = nullptr;
    free_slot(sl);
    return fail(LFC_E_NOMEM, "lfc_batch_render: device staging");
  }
  sl.cap = cap;
  return LFC_OK;
}

// Marks the slot's table in use until the work just queued on s (the copy
// and the launches that read it) has finished.  If the mark cannot be
// recorded, waits for s instead, so that the slot is free again.
lfc_status release_slot(Slot &sl, lfc_status st, hipStream_t s, const char *who) {
  if (hipEventRecord(sl.done, s) == hipSuccess) {
    sl.used = true;
    return st;
  }
  (void)hipStreamSynchronize(s);
  return st != LFC_OK ? st : fail(LFC_E_HIP, std::string(who) + ": event record");
}

}  // namespace

extern "C" lfc_status lfc_batch_create(lfc_batch **out) {
  if (!out) return fail(LFC_E_INVALID, "lfc_batch_create: null out");
  *out = nullptr;
  lfc_batch *b = new (std::nothrow) lfc_batch;
  if (!b) return fail(LFC_E_NOMEM, "lfc_batch_create: out of host memory");
  if (hipGetDevice(&b->device) != hipSuccess) {
    delete b;
    return fail(LFC_E_HIP, "lfc_batch_create: no current device");
  }
  for (Slot &sl : b->slot) {
    if (hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) {
      (void)lfc_batch_destroy(b);
      return fail(LFC_E_HIP, "lfc_batch_create: event");
    }
  }
  if (hipMalloc(reinterpret_cast<void **>(&b->d_err), sizeof(int32_t)) != hipSuccess ||
      hipMemset(b->d_err, 0, sizeof(int32_t)) != hipSuccess ||
      hipMalloc(reinterpret_cast<void **>(&b->d_ctr), kSlots * kCtrStride * sizeof(uint32_t)) != hipSuccess ||
      hipMemset(b->d_ctr, 0, kSlots * kCtrStride * sizeof(uint32_t)) != hipSuccess) {
    (void)lfc_batch_destroy(b);
    return fail(LFC_E_NOMEM, "lfc_batch_create: error flag");
  }
  *out = b;
  return LFC_OK;
}

extern "C" lfc_status lfc_batch_destroy(lfc_batch *b) {
  if (!b) return LFC_OK;
  for (Slot &sl : b->slot) {
    if (sl.done) {
      if (sl.used) (void)hipEventSynchronize(sl.done);
      (void)hipEventDestroy(sl.done);
    }
    free_slot(sl);
  }
  for (Scratch &sc : b->scratch) {
    if (sc.used) (void)hipEventSynchronize(sc.done);
    if (sc.done) (void)hipEventDestroy(sc.done);
    if (sc.buf) (void)hipFree(sc.buf);
  }
  if (b->d_err) (void)hipFree(b->d_err);
  if (b->d_ctr) (void)hipFree(b->d_ctr);
  delete b;
  return LFC_OK;
}

namespace {

// The context's scratch for lf's decoded views: an existing buffer that
// holds them, else a new one; nullptr if there is no room (the caller then
// renders that light field by tiles).
Scratch *get_scratch(lfc_batch *b, const lfc_lf *lf) {
  const size_t need = lfc::lf_rgb_bytes(lf);
  for (Scratch &sc : b->scratch)
    if (sc.lf == lf && sc.bytes >= need) return &sc;
  Scratch sc;
  sc.lf = lf;
  sc.bytes = need;
  if (hipMalloc(&sc.buf, need) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  if (hipEventCreateWithFlags(&sc.done, hipEventDisableTiming) != hipSuccess) {
    (void)hipFree(sc.buf);
    return nullptr;
  }
  b->scratch.push_back(sc);
  return &b->scratch.back();
}

size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

// A batch resolved on the host: which path each light field takes, the
// decoded-view buffers, and where each part of its table goes.  The table:
// tile requests grouped by block size; per block size the colour decode's
// light-field records and first work items; the view masks; the
// interpolated requests.
struct BatchLayout {
  struct Group {
    int count = 0, max_tiles = 0;   // tile requests
    size_t lds = 0;
    size_t at_tiles = 0;
    std::vector<int> lf;            // colour-decoded light fields of this block size
    bool keys = true;
    size_t rgb_lds = 0;
    int items = 0;
    size_t at_args = 0, at_first = 0;
  } grp[9];
  std::vector<char> tiles;          // packed tile requests, in table order
  std::vector<Scratch *> scr;       // per light field: its decoded views (colour path) or null (tiles)
  std::vector<size_t> at_mask;
  size_t at_interp = 0, bytes = 0;
  int n_interp = 0, max_wo = 0, max_ho = 0;
};

// Validates a batch and lays out its table (see BatchLayout); with
// check_outs false the output pointers are trusted to hold their results
// (the server's pool offsets, sized when admitted); allow_rgb (null: every
// light field) limits the colour path.
lfc_status plan_batch(lfc_batch *b, const lfc_lf *const *lfs, int32_t n_lf, const lfc_render_request *reqs, int32_t n,
                      float *const *d_outs, bool check_outs, const char *allow_rgb, BatchLayout &L,
                      const char *who) {
  if (!lfs || n_lf < 1 || !reqs || !d_outs) return fail(LFC_E_INVALID, std::string(who) + ": null array");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != b->device)
    return fail(LFC_E_INVALID, std::string(who) + ": the current device is not the batch's");
  for (int i = 0; i < n_lf; i++)
    if (!lfs[i] || lfc::lf_device(lfs[i]) != dev)
      return fail(LFC_E_INVALID, std::string(who) + ": null handle or handle of another device");
  // requests checked; output pixels per light field
  std::vector<double> px(n_lf, 0.0);
  for (int i = 0; i < n; i++) {
    const lfc_render_request &r = reqs[i];
    if (r.lf < 0 || r.lf >= n_lf) return fail(LFC_E_INVALID, std::string(who) + ": request lf index out of range");
    if (r.out_w < 1 || r.out_h < 1 || r.out_w > 16384 || r.out_h > 16384)
      return fail(LFC_E_INVALID, std::string(who) + ": out_w and out_h must be 1..16384");
    if (!d_outs[i] || reinterpret_cast<uintptr_t>(d_outs[i]) % 4)
      return fail(LFC_E_INVALID, std::string(who) + ": null or unaligned output pointer");
    if (check_outs)
      if (lfc_status st = lfc::device_buffer(d_outs[i], (size_t)3 * r.out_w * r.out_h * sizeof(float), 4, who,
                                             "d_outs[i]"))
        return st;
    px[(size_t)r.lf] += (double)r.out_w * r.out_h;
  }
  // a light field whose requests cover about as many pixels as it holds is
  // decoded once (the views they read, as 8-bit RGB) and interpolated; the
  // others render by tiles, each tile decoding its own footprint
  L.scr.assign((size_t)n_lf, nullptr);
  for (int l = 0; l < n_lf; l++)
    if (px[(size_t)l] > 0.0 && (!allow_rgb || allow_rgb[l]) && lfc::lf_rgb_batchable(lfs[l], px[(size_t)l]))
      L.scr[(size_t)l] = get_scratch(b, lfs[l]);
  const size_t rb = lfc::render_req_bytes(), ab = lfc::rgb_args_bytes(), ib = lfc::interp_req_bytes();
  std::vector<char> packed((size_t)n * rb);
  std::vector<int> bs(n, 0);
  for (int i = 0; i < n; i++) {
    const lfc_render_request &r = reqs[i];
    if (L.scr[(size_t)r.lf]) {
      L.n_interp++;
      L.max_wo = std::max(L.max_wo, r.out_w);
      L.max_ho = std::max(L.max_ho, r.out_h);
      continue;
    }
    int block = 0, nt = 0;
    size_t lds = 0;
    if (lfc_status st = lfc::render_req_fill(lfs[r.lf], r.view, r.out_w, r.out_h, d_outs[i], &packed[(size_t)i * rb],
                                             &block, &nt, &lds))
      return st;
    bs[i] = block;
    BatchLayout::Group &gp = L.grp[block];
    gp.count++;
    gp.max_tiles = std::max(gp.max_tiles, nt);
    gp.lds = std::max(gp.lds, lds);
  }
  for (int block : {2, 4, 8})
    if (L.grp[block].count > 65535)
      return fail(LFC_E_INVALID, std::string(who) + ": more than 65535 requests of one block size");
  size_t at = 0;
  for (int block : {2, 4, 8}) {
    L.grp[block].at_tiles = at;
    for (int i = 0; i < n; i++)
      if (bs[i] == block) {
        L.tiles.insert(L.tiles.end(), packed.begin() + (ptrdiff_t)((size_t)i * rb),
                       packed.begin() + (ptrdiff_t)((size_t)(i + 1) * rb));
        at += rb;
      }
  }
  at = align16(at);
  for (int l = 0; l < n_lf; l++)
    if (L.scr[(size_t)l]) L.grp[lfc::lf_block(lfs[l])].lf.push_back(l);
  for (int block : {2, 4, 8}) {
    BatchLayout::Group &gp = L.grp[block];
    if (gp.lf.empty()) continue;
    for (int l : gp.lf) gp.keys = gp.keys && lfc::rgb_keys_fit(lfs[l]);
    for (int l : gp.lf) gp.rgb_lds = std::max(gp.rgb_lds, lfc::rgb_lds_bytes(lfs[l], gp.keys));
    for (int l : gp.lf) gp.items += lfc::lf_rgb_items(lfs[l]);
    gp.at_args = at;
    at = align16(at + gp.lf.size() * ab);
    gp.at_first = at;
    at = align16(at + 4 * (gp.lf.size() + 1));
  }
  L.at_mask.assign((size_t)n_lf, 0);
  for (int l = 0; l < n_lf; l++)
    if (L.scr[(size_t)l]) {
      L.at_mask[(size_t)l] = at;
      at = align16(at + 4 * (size_t)((lfc::lf_views(lfs[l]) + 31) / 32));
    }
  L.at_interp = at;
  L.bytes = align16(at + (size_t)L.n_interp * ib);
  return LFC_OK;
}

// Writes a planned batch's table into host (bytes L.bytes) for a device
// copy at dev.
void fill_batch(const BatchLayout &L, const lfc_lf *const *lfs, int32_t n_lf, const lfc_render_request *reqs,
                int32_t n, float *const *d_outs, char *host, const char *dev) {
  const size_t ab = lfc::rgb_args_bytes(), ib = lfc::interp_req_bytes();
  std::memset(host, 0, L.bytes);
  if (!L.tiles.empty()) std::memcpy(host, L.tiles.data(), L.tiles.size());
  for (int block : {2, 4, 8}) {
    const BatchLayout::Group &gp = L.grp[block];
    int32_t *first = reinterpret_cast<int32_t *>(host + gp.at_first);
    int items = 0;
    for (size_t k = 0; k < gp.lf.size(); k++) {
      const int l = gp.lf[k];
      lfc::rgb_args_fill(lfs[l], gp.keys, static_cast<uint32_t *>(L.scr[(size_t)l]->buf),
                         reinterpret_cast<const uint32_t *>(dev + L.at_mask[(size_t)l]), host + gp.at_args + k * ab);
      first[k] = items;
      items += lfc::lf_rgb_items(lfs[l]);
    }
    if (!gp.lf.empty()) first[gp.lf.size()] = items;
  }
  int k = 0;
  for (int i = 0; i < n; i++) {
    const lfc_render_request &r = reqs[i];
    if (!L.scr[(size_t)r.lf]) continue;
    lfc::need_mask_host(lfs[r.lf], r.view, reinterpret_cast<uint32_t *>(host + L.at_mask[(size_t)r.lf]));
    lfc::interp_req_fill(lfs[r.lf], static_cast<uint32_t *>(L.scr[(size_t)r.lf]->buf), r.view, r.out_w, r.out_h,
                         d_outs[i], host + L.at_interp + (size_t)k * ib);
    k++;
  }
  (void)n_lf;
}

// The launches of a batch whose table is at dev: tile groups, then the
// colour decode of each block size (persistent, counters ctr[2]), then the
// interpolation.  No copies, memsets or event operations: a stream capture
// of it is a graph of kernels only.
lfc_status launch_batch(const BatchLayout &L, const char *dev, uint32_t *ctr, hipStream_t s) {
  lfc_status st = LFC_OK;
  for (int block : {2, 4, 8}) {
    const BatchLayout::Group &gp = L.grp[block];
    if (gp.count && st == LFC_OK)
      st = lfc::render_multi_launch(block, dev + gp.at_tiles, gp.count, gp.max_tiles, gp.lds, s);
  }
  for (int block : {2, 4, 8}) {
    const BatchLayout::Group &gp = L.grp[block];
    if (gp.lf.empty() || st != LFC_OK) continue;
    st = lfc::rgb_multi_launch(block, gp.keys, dev + gp.at_args, reinterpret_cast<const int32_t *>(dev + gp.at_first),
                               (int)gp.lf.size(), gp.items, gp.rgb_lds, ctr, s);
  }
  if (st == LFC_OK && L.n_interp) st = lfc::interp_multi_launch(dev + L.at_interp, L.n_interp, L.max_wo, L.max_ho, s);
  return st;
}

// lfc_batch_render (see plan_batch for check_outs and allow_rgb).
lfc_status batch_render(lfc_batch *b, const lfc_lf *const *lfs, int32_t n_lf, const lfc_render_request *reqs,
                        int32_t n, float *const *d_outs, hipStream_t s, bool check_outs,
                        const char *allow_rgb = nullptr) {
  const char *who = "lfc_batch_render";
  if (!b) return fail(LFC_E_INVALID, "lfc_batch_render: null batch");
  if (n < 0) return fail(LFC_E_INVALID, "lfc_batch_render: n < 0");
  if (n == 0) return LFC_OK;
  BatchLayout L;
  if (lfc_status st = plan_batch(b, lfs, n_lf, reqs, n, d_outs, check_outs, allow_rgb, L, who)) return st;
  Slot &sl = b->slot[b->next];
  if (lfc_status st = grow_slot(sl, L.bytes)) return st;
  // the kernels that read the slot's previous table must have finished
  if (sl.used && hipEventSynchronize(sl.done) != hipSuccess) return fail(LFC_E_HIP, "lfc_batch_render: event wait");
  sl.used = false;
  fill_batch(L, lfs, n_lf, reqs, n, d_outs, sl.host, sl.dev);
  if (hipMemcpyAsync(sl.dev, sl.host, L.bytes, hipMemcpyHostToDevice, s) != hipSuccess)
    return fail(LFC_E_HIP, std::string(who) + ": copy of the request table");
  uint32_t *ctr = b->d_ctr + (size_t)b->next * kCtrStride;
  b->next = (b->next + 1) % kSlots;
  // a decoded-views buffer is rewritten only after the launches of an
  // earlier batch that read it (on any stream) have finished
  lfc_status st = LFC_OK;
  for (int l = 0; l < n_lf && st == LFC_OK; l++)
    if (L.scr[(size_t)l] && L.scr[(size_t)l]->used && hipStreamWaitEvent(s, L.scr[(size_t)l]->done, 0) != hipSuccess)
      st = fail(LFC_E_HIP, std::string(who) + ": wait for an earlier use of the decoded views");
  if (st == LFC_OK) st = launch_batch(L, sl.dev, ctr, s);
  for (int l = 0; l < n_lf; l++)
    if (L.scr[(size_t)l]) {
      if (hipEventRecord(L.scr[(size_t)l]->done, s) == hipSuccess) {
        L.scr[(size_t)l]->used = true;
      } else {
        (void)hipStreamSynchronize(s);
        L.scr[(size_t)l]->used = false;
        if (st == LFC_OK) st = fail(LFC_E_HIP, std::string(who) + ": event record");
      }
    }
  return release_slot(sl, st, s, who);
}

}  // namespace

extern "C" lfc_status lfc_batch_render(lfc_batch *b, const lfc_lf *const *lfs, int32_t n_lf,
                                       const lfc_render_request *reqs, int32_t n, float *const *d_outs,
                                       hipStream_t s) {
  return batch_render(b, lfs, n_lf, reqs, n, d_outs, s, true);
}

// A batch fixed once: its table on the device, its decoded-view buffers
// (in a context of its own) and the colour decode's counters, and with a
// graph its launches captured once.
struct lfc_batch_plan {
  lfc_batch *b = nullptr;
  BatchLayout L;
  char *dev = nullptr;
  uint32_t *ctr = nullptr;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" void lfc_batch_plan_destroy(lfc_batch_plan *p) {
  if (!p) return;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->cap) (void)hipStreamDestroy(p->cap);
  if (p->dev || p->ctr) (void)hipDeviceSynchronize();
  if (p->dev) (void)hipFree(p->dev);
  if (p->ctr) (void)hipFree(p->ctr);
  (void)lfc_batch_destroy(p->b);
  delete p;
}

extern "C" lfc_status lfc_batch_plan_create(const lfc_lf *const *lfs, int32_t n_lf, const lfc_render_request *reqs,
                                            int32_t n, float *const *d_outs, int32_t graph, lfc_batch_plan **out) {
  const char *who = "lfc_batch_plan_create";
  if (!out) return fail(LFC_E_INVALID, "lfc_batch_plan_create: null result");
  *out = nullptr;
  if (n < 1) return fail(LFC_E_INVALID, "lfc_batch_plan_create: n must be at least 1");
  lfc_batch_plan *p = new (std::nothrow) lfc_batch_plan;
  if (!p) return fail(LFC_E_NOMEM, "lfc_batch_plan_create: out of host memory");
  lfc_status st = lfc_batch_create(&p->b);
  if (st == LFC_OK) st = plan_batch(p->b, lfs, n_lf, reqs, n, d_outs, true, nullptr, p->L, who);
  std::vector<char> host;
  if (st == LFC_OK) {
    host.resize(p->L.bytes);
    if (hipMalloc(reinterpret_cast<void **>(&p->dev), p->L.bytes) != hipSuccess) {
      p->dev = nullptr;
      st = fail(LFC_E_NOMEM, "lfc_batch_plan_create: request table");
    } else if (hipMalloc(reinterpret_cast<void **>(&p->ctr), 2 * sizeof(uint32_t)) != hipSuccess) {
      p->ctr = nullptr;
      st = fail(LFC_E_NOMEM, "lfc_batch_plan_create: counters");
    }
  }
  if (st == LFC_OK) {
    fill_batch(p->L, lfs, n_lf, reqs, n, d_outs, host.data(), p->dev);
    if (hipMemcpy(p->dev, host.data(), p->L.bytes, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(p->ctr, 0, 2 * sizeof(uint32_t)) != hipSuccess)
      st = fail(LFC_E_HIP, "lfc_batch_plan_create: copy of the request table");
  }
  if (st == LFC_OK && graph) {
    if (hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking) != hipSuccess) {
      p->cap = nullptr;
      st = fail(LFC_E_HIP, "lfc_batch_plan_create: capture stream");
    } else if (hipStreamBeginCapture(p->cap, hipStreamCaptureModeRelaxed) != hipSuccess) {
      st = fail(LFC_E_HIP, "lfc_batch_plan_create: begin capture");
    } else {
      st = launch_batch(p->L, p->dev, p->ctr, p->cap);
      hipGraph_t g = nullptr;
      const hipError_t he = hipStreamEndCapture(p->cap, &g);
      p->graph = g;
      if (st == LFC_OK && (he != hipSuccess || !g)) st = fail(LFC_E_HIP, "lfc_batch_plan_create: end capture");
      if (st == LFC_OK && hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess) {
        p->exec = nullptr;
        st = fail(LFC_E_HIP, "lfc_batch_plan_create: graph instantiation");
      }
    }
  }
  if (st != LFC_OK) {
    lfc_batch_plan_destroy(p);
    return st;
  }
  *out = p;
  return LFC_OK;
}

extern "C" lfc_status lfc_batch_plan_launch(lfc_batch_plan *p, hipStream_t s) {
  if (!p) return fail(LFC_E_INVALID, "lfc_batch_plan_launch: null plan");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != p->b->device)
    return fail(LFC_E_INVALID, "lfc_batch_plan_launch: the current device is not the plan's");
  if (p->exec) {
    if (hipGraphLaunch(p->exec, s) != hipSuccess) return fail(LFC_E_HIP, "lfc_batch_plan_launch: graph launch");
    return LFC_OK;
  }
  return launch_batch(p->L, p->dev, p->ctr, s);
}

extern "C" lfc_status lfc_batch_plan_info(const lfc_batch_plan *p, int32_t *n_decoded_lf, int32_t *graph) {
  if (!p || !n_decoded_lf || !graph) return fail(LFC_E_INVALID, "lfc_batch_plan_info: null argument");
  int k = 0;
  for (const Scratch *sc : p->L.scr) k += sc != nullptr;
  *n_decoded_lf = k;
  *graph = p->exec != nullptr;
  return LFC_OK;
}

extern "C" lfc_status lfc_batch_decode(lfc_batch *b, const lfc_lf *const *lfs, int32_t n_lf, const int32_t *d_req,
                                       int64_t n, int16_t *d_out, hipStream_t s) {
  if (!b) return fail(LFC_E_INVALID, "lfc_batch_decode: null batch");
  if (n < 0) return fail(LFC_E_INVALID, "lfc_batch_decode: n < 0");
  if (n == 0) return LFC_OK;
  if (!lfs || n_lf < 1 || !d_req || !d_out) return fail(LFC_E_INVALID, "lfc_batch_decode: null argument");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != b->device)
    return fail(LFC_E_INVALID, "lfc_batch_decode: the current device is not the batch's");
  int block = 0;
  for (int i = 0; i < n_lf; i++) {
    if (!lfs[i] || lfc::lf_device(lfs[i]) != dev)
      return fail(LFC_E_INVALID, "lfc_batch_decode: null handle or handle of another device");
    if (i == 0) block = lfc::lf_block(lfs[i]);
    else if (lfc::lf_block(lfs[i]) != block)
      return fail(LFC_E_UNSUPPORTED, "lfc_batch_decode: the light fields of one call must share the block size");
  }
  if (lfc_status st = lfc::device_buffer(d_req, (size_t)n * 3 * sizeof(int32_t), 4, "lfc_batch_decode", "d_req"))
    return st;
  if (lfc_status st = lfc::device_buffer(d_out, (size_t)n * 3 * block * block * sizeof(int16_t), 16,
                                         "lfc_batch_decode", "d_out"))
    return st;
  const size_t tb = lfc::lf_table_bytes();
  Slot &sl = b->slot[b->next];
  if (lfc_status st = grow_slot(sl, (size_t)n_lf * tb)) return st;
  if (sl.used && hipEventSynchronize(sl.done) != hipSuccess) return fail(LFC_E_HIP, "lfc_batch_decode: event wait");
  sl.used = false;
  for (int i = 0; i < n_lf; i++) lfc::lf_table_fill(lfs[i], sl.host + (size_t)i * tb);
  if (hipMemcpyAsync(sl.dev, sl.host, (size_t)n_lf * tb, hipMemcpyHostToDevice, s) != hipSuccess)
    return fail(LFC_E_HIP, "lfc_batch_decode: copy of the light-field table");
  b->next = (b->next + 1) % kSlots;
  return release_slot(sl, lfc::decode_multi_launch(block, sl.dev, n_lf, d_req, n, d_out, b->d_err, s), s,
                      "lfc_batch_decode");
}

extern "C" lfc_status lfc_batch_check(lfc_batch *b, hipStream_t s) {
  if (!b) return fail(LFC_E_INVALID, "lfc_batch_check: null batch");
  int32_t flag = 0;
  if (hipStreamSynchronize(s) != hipSuccess || hipMemcpy(&flag, b->d_err, 4, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemset(b->d_err, 0, 4) != hipSuccess)
    return fail(LFC_E_HIP, "lfc_batch_check: reading the error flag");
  if (flag) return fail(LFC_E_INVALID, "lfc_batch_decode: a request was out of range (zeros written)");
  return LFC_OK;
}

// ---------------------------------------------------------------------------
// serving loop
// ---------------------------------------------------------------------------

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

// First-fit allocator over [0, size) with coalescing, 256-byte granules.
class Pool {
 public:
  void reset(size_t size) {
    free_.clear();
    free_[0] = size;
    used_ = 0;
  }
  bool alloc(size_t bytes, size_t *off) {
    bytes = (bytes + 255) & ~(size_t)255;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes, at = it->first + bytes;
      free_.erase(it);
      if (rest) free_[at] = rest;
      used_ += bytes;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = (bytes + 255) & ~(size_t)255;
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }

 private:
  std::map<size_t, size_t> free_;
  size_t used_ = 0;
};

enum class State { Queued, Running, Done, Failed };

struct Ticket {
  lfc_render_request req;
  size_t bytes = 0, off = 0;
  State state = State::Queued;
  lfc_status status = LFC_OK;
  bool discard = false;        // released by the engine on completion (replay)
  double *latency_out = nullptr;
  Clock::time_point t_submit, t_done;
};

struct Lane {                  // one launch slot: a stream, its batch context, its batch in flight
  hipStream_t stream = nullptr;
  lfc_batch *batch = nullptr;
  hipEvent_t done = nullptr;
  std::vector<uint64_t> running;
};

}  // namespace

struct lfc_server {
  std::vector<const lfc_lf *> lfs;
  std::vector<char> allow_rgb;   // per light field: its batches may use the colour path (memory granted)
  lfc_server_config cfg{};
  int device = 0;
  char *d_pool = nullptr;
  Pool pool;
  std::vector<Lane> lanes;
  std::mutex mu;
  std::condition_variable cv_engine, cv_done;
  std::deque<uint64_t> queue;
  std::unordered_map<uint64_t, Ticket> tickets;
  uint64_t next_ticket = 1;
  bool stop = false;
  int64_t replay_left = 0;
  uint64_t releases = 0;     // pool releases by clients, to wake a blocked engine
  uint64_t last_blocked = 0; // the last queue head counted as waiting for room
  lfc_server_stats stats{};
  std::thread engine;
  std::string engine_error;
};

namespace {

size_t result_bytes(const lfc_render_request &r) { return (size_t)3 * r.out_w * r.out_h * sizeof(float); }

// Completes the lane's batch (its event has fired).  Caller holds mu.
void finish_lane(lfc_server *sv, Lane &ln, lfc_status st) {
  const Clock::time_point now = Clock::now();
  for (uint64_t id : ln.running) {
    auto it = sv->tickets.find(id);
    if (it == sv->tickets.end()) continue;
    Ticket &t = it->second;
    t.t_done = now;
    t.status = st;
    t.state = st == LFC_OK ? State::Done : State::Failed;
    sv->stats.completed++;
    if (t.discard) {
      if (t.latency_out) *t.latency_out = ms_between(t.t_submit, now);
      sv->pool.release(t.off, t.bytes);
      sv->tickets.erase(it);
      sv->replay_left--;
    }
  }
  ln.running.clear();
  sv->cv_done.notify_all();
}

void engine_loop(lfc_server *sv) {
  (void)hipSetDevice(sv->device);
  std::vector<const lfc_lf *> &lfs = sv->lfs;
  std::vector<lfc_render_request> reqs;
  std::vector<float *> outs;
  std::vector<uint64_t> ids;
  std::unique_lock<std::mutex> lk(sv->mu);
  for (;;) {
    // completions
    bool busy = false;
    for (Lane &ln : sv->lanes) {
      if (ln.running.empty()) continue;
      const hipError_t q = hipEventQuery(ln.done);
      if (q == hipSuccess) finish_lane(sv, ln, LFC_OK);
      else if (q == hipErrorNotReady) busy = true;
      else finish_lane(sv, ln, LFC_E_HIP);
    }
    // admission and launch on a free lane
    Lane *free_lane = nullptr;
    for (Lane &ln : sv->lanes)
      if (ln.running.empty()) {
        free_lane = &ln;
        break;
      }
    bool blocked = false;   // the head of the queue waits for pool room
    if (free_lane && !sv->queue.empty()) {
      reqs.clear();
      outs.clear();
      ids.clear();
      while (!sv->queue.empty() && (int)ids.size() < sv->cfg.max_batch) {
        Ticket &t = sv->tickets[sv->queue.front()];
        if (!sv->pool.alloc(t.bytes, &t.off)) {
          if (ids.empty()) {
            if (sv->last_blocked != sv->queue.front()) sv->stats.admission_waits++;
            sv->last_blocked = sv->queue.front();
            blocked = true;
          }
          break;
        }
        t.state = State::Running;
        ids.push_back(sv->queue.front());
        reqs.push_back(t.req);
        outs.push_back(reinterpret_cast<float *>(sv->d_pool + t.off));
        sv->queue.pop_front();
      }
      if (!ids.empty()) {
        Lane &ln = *free_lane;
        ln.running = ids;
        sv->stats.batches++;
        sv->stats.max_batch_seen = std::max<int64_t>(sv->stats.max_batch_seen, (int64_t)ids.size());
        lk.unlock();
        lfc_status st = batch_render(ln.batch, lfs.data(), (int32_t)lfs.size(), reqs.data(), (int32_t)reqs.size(),
                                     outs.data(), ln.stream, false, sv->allow_rgb.data());
        if (st == LFC_OK && hipEventRecord(ln.done, ln.stream) != hipSuccess) st = LFC_E_HIP;
        if (st != LFC_OK) {
          // a failure after some of the batch's launches were queued (one per
          // block size): those still write into the batch's pool regions, so
          // the regions are freed only once the lane's stream has drained
          sv->engine_error = lfc_last_error();
          (void)hipStreamSynchronize(ln.stream);
        }
        lk.lock();
        if (st != LFC_OK) finish_lane(sv, ln, st);
        continue;
      }
    }
    if (busy) {
      // launches in flight: poll their events without holding the lock
      lk.unlock();
      std::this_thread::yield();
      lk.lock();
      continue;
    }
    if (sv->stop && (sv->queue.empty() || blocked)) {
      // nothing in flight: whatever is still queued can never be admitted
      for (uint64_t id : sv->queue) {
        Ticket &t = sv->tickets[id];
        t.state = State::Failed;
        t.status = LFC_E_INVALID;
        if (t.discard) sv->replay_left--;
      }
      sv->queue.clear();
      sv->engine_error = "the server stopped before the request was admitted";
      sv->cv_done.notify_all();
      break;
    }
    const uint64_t seen = sv->releases;
    sv->cv_engine.wait(lk, [&] {
      return sv->stop || (!sv->queue.empty() && !blocked) || sv->releases != seen;
    });
  }
}

lfc_status submit_locked(lfc_server *sv, const lfc_render_request &r, bool discard, double *lat_out, uint64_t *id) {
  if (r.lf < 0 || r.lf >= (int32_t)sv->lfs.size())
    return fail(LFC_E_INVALID, "lfc_server_submit: lf index out of range");
  if (r.out_w < 1 || r.out_h < 1 || r.out_w > 16384 || r.out_h > 16384)
    return fail(LFC_E_INVALID, "lfc_server_submit: out_w and out_h must be 1..16384");
  const size_t bytes = result_bytes(r);
  if (((bytes + 255) & ~(size_t)255) > (size_t)sv->cfg.out_pool_bytes)
    return fail(LFC_E_INVALID, "lfc_server_submit: result larger than the output pool");
  if (sv->cfg.max_queue > 0 && (int64_t)sv->queue.size() >= sv->cfg.max_queue)
    return fail(LFC_E_NOMEM, "lfc_server_submit: the queue is full (max_queue requests wait for admission)");
  const uint64_t t_id = sv->next_ticket++;
  Ticket &t = sv->tickets[t_id];
  t.req = r;
  t.bytes = bytes;
  t.discard = discard;
  t.latency_out = lat_out;
  t.t_submit = Clock::now();
  sv->queue.push_back(t_id);
  sv->stats.submitted++;
  if (id) *id = t_id;
  return LFC_OK;
}

}  // namespace

extern "C" lfc_status lfc_server_create(const lfc_lf *const *lfs, int32_t n_lf, const lfc_server_config *cfg,
                                        lfc_server **out) {
  if (!out) return fail(LFC_E_INVALID, "lfc_server_create: null out");
  *out = nullptr;
  if (!lfs || n_lf < 1 || !cfg) return fail(LFC_E_INVALID, "lfc_server_create: null argument or no light field");
  if (cfg->max_batch < 1 || cfg->max_batch > 65535 || cfg->streams < 1 || cfg->streams > 8 ||
      cfg->out_pool_bytes < 256 || cfg->max_queue < 0 || cfg->device_bytes_cap < 0)
    return fail(LFC_E_INVALID, "lfc_server_create: max_batch 1..65535, streams 1..8, out_pool_bytes >= 256, "
                               "max_queue and device_bytes_cap >= 0");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(LFC_E_HIP, "lfc_server_create: no current device");
  for (int i = 0; i < n_lf; i++)
    if (!lfs[i] || lfc::lf_device(lfs[i]) != dev)
      return fail(LFC_E_INVALID, "lfc_server_create: null handle or handle of another device");
  lfc_server *sv = new (std::nothrow) lfc_server;
  if (!sv) return fail(LFC_E_NOMEM, "lfc_server_create: out of host memory");
  sv->lfs.assign(lfs, lfs + n_lf);
  sv->cfg = *cfg;
  sv->device = dev;
  // memory admission: the resident light fields and the output pool first,
  // then the colour path's decoded-view buffers (one per light field and
  // stream), light field by light field, while they fit
  sv->allow_rgb.assign((size_t)n_lf, 1);
  if (cfg->device_bytes_cap > 0) {
    int64_t used = cfg->out_pool_bytes;
    for (int i = 0; i < n_lf; i++) {
      lfc_info_t info;
      (void)lfc_info(lfs[i], &info);
      used += (int64_t)info.device_bytes;
    }
    if (used > cfg->device_bytes_cap) {
      delete sv;
      return fail(LFC_E_NOMEM, "lfc_server_create: the light fields and the output pool need " + std::to_string(used) +
                                   " device bytes, more than device_bytes_cap");
    }
    for (int i = 0; i < n_lf; i++) {
      const int64_t need = (int64_t)cfg->streams * (int64_t)lfc::lf_rgb_bytes(lfs[i]);
      if (used + need <= cfg->device_bytes_cap) used += need;
      else sv->allow_rgb[(size_t)i] = 0;
    }
  }
  if (hipMalloc(reinterpret_cast<void **>(&sv->d_pool), (size_t)cfg->out_pool_bytes) != hipSuccess) {
    delete sv;
    return fail(LFC_E_NOMEM, "lfc_server_create: output pool");
  }
  sv->pool.reset((size_t)cfg->out_pool_bytes);
  sv->lanes.resize(cfg->streams);
  for (Lane &ln : sv->lanes) {
    if (hipStreamCreateWithFlags(&ln.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ln.done, hipEventDisableTiming) != hipSuccess || lfc_batch_create(&ln.batch)) {
      sv->stop = true;
      (void)lfc_server_destroy(sv);
      return fail(LFC_E_HIP, "lfc_server_create: stream, event or batch context");
    }
  }
  sv->engine = std::thread(engine_loop, sv);
  *out = sv;
  return LFC_OK;
}

extern "C" lfc_status lfc_server_submit(lfc_server *sv, const lfc_render_request *req, uint64_t *ticket) {
  if (!sv || !req || !ticket) return fail(LFC_E_INVALID, "lfc_server_submit: null argument");
  std::lock_guard<std::mutex> lk(sv->mu);
  if (lfc_status st = submit_locked(sv, *req, false, nullptr, ticket)) return st;
  sv->cv_engine.notify_one();
  return LFC_OK;
}

extern "C" lfc_status lfc_server_wait(lfc_server *sv, uint64_t ticket, int32_t timeout_ms, const float **d_img,
                                      double *latency_ms) {
  if (!sv) return fail(LFC_E_INVALID, "lfc_server_wait: null server");
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->tickets.find(ticket);
  if (it == sv->tickets.end() || it->second.discard) return fail(LFC_E_INVALID, "lfc_server_wait: unknown ticket");
  auto ready = [&] {
    const State s = sv->tickets[ticket].state;
    return s == State::Done || s == State::Failed;
  };
  if (timeout_ms < 0) sv->cv_done.wait(lk, ready);
  else if (!sv->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready))
    return fail(LFC_E_INVALID, "lfc_server_wait: timed out");
  const Ticket &t = sv->tickets[ticket];
  if (t.state == State::Failed)
    return fail(t.status, "lfc_server_wait: the request's launch failed: " + sv->engine_error);
  if (d_img) *d_img = reinterpret_cast<const float *>(sv->d_pool + t.off);
  if (latency_ms) *latency_ms = ms_between(t.t_submit, t.t_done);
  return LFC_OK;
}

extern "C" lfc_status lfc_server_release(lfc_server *sv, uint64_t ticket) {
  if (!sv) return fail(LFC_E_INVALID, "lfc_server_release: null server");
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->tickets.find(ticket);
  if (it == sv->tickets.end() || it->second.discard) return fail(LFC_E_INVALID, "lfc_server_release: unknown ticket");
  Ticket &t = it->second;
  if (t.state == State::Queued || t.state == State::Running)
    return fail(LFC_E_INVALID, "lfc_server_release: the request has not completed");
  sv->pool.release(t.off, t.bytes);
  sv->tickets.erase(it);
  sv->releases++;
  sv->cv_engine.notify_one();
  return LFC_OK;
}

extern "C" lfc_status lfc_server_replay(lfc_server *sv, const lfc_render_request *reqs, const double *arrival_ms,
                                        int32_t n, double *latency_ms) {
  if (!sv || n < 0 || (n > 0 && (!reqs || !arrival_ms || !latency_ms)))
    return fail(LFC_E_INVALID, "lfc_server_replay: null argument or n < 0");
  for (int i = 0; i < n; i++) {
    if (i && arrival_ms[i] < arrival_ms[i - 1]) return fail(LFC_E_INVALID, "lfc_server_replay: arrivals not sorted");
    const lfc_render_request &r = reqs[i];
    if (r.lf < 0 || r.lf >= (int32_t)sv->lfs.size() || r.out_w < 1 || r.out_h < 1 || r.out_w > 16384 ||
        r.out_h > 16384 || ((result_bytes(r) + 255) & ~(size_t)255) > (size_t)sv->cfg.out_pool_bytes)
      return fail(LFC_E_INVALID, "lfc_server_replay: request out of range");
  }
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->replay_left += n;
  }
  const Clock::time_point t0 = Clock::now();
  for (int i = 0; i < n; i++) {
    const Clock::time_point due = t0 + std::chrono::duration_cast<Clock::duration>(
                                           std::chrono::duration<double, std::milli>(arrival_ms[i]));
    for (;;) {
      const Clock::time_point now = Clock::now();
      if (now >= due) break;
      if (due - now > std::chrono::microseconds(200)) std::this_thread::sleep_for(due - now - std::chrono::microseconds(100));
      else std::this_thread::yield();
    }
    std::lock_guard<std::mutex> lk(sv->mu);
    lfc_status st = submit_locked(sv, reqs[i], true, &latency_ms[i], nullptr);
    if (st == LFC_E_NOMEM) {   // refused: the queue is full
      latency_ms[i] = -1.0;
      sv->replay_left--;
      sv->cv_done.notify_all();
      continue;
    }
    if (st != LFC_OK) return st;
    // latency counts from the scheduled arrival, so a late submit is not hidden
    sv->tickets[sv->next_ticket - 1].t_submit = due;
    sv->cv_engine.notify_one();
  }
  std::unique_lock<std::mutex> lk(sv->mu);
  sv->cv_done.wait(lk, [&] { return sv->replay_left <= 0; });
  return LFC_OK;
}

extern "C" lfc_status lfc_server_get_stats(lfc_server *sv, lfc_server_stats *st) {
  if (!sv || !st) return fail(LFC_E_INVALID, "lfc_server_get_stats: null argument");
  std::lock_guard<std::mutex> lk(sv->mu);
  *st = sv->stats;
  st->pool_bytes_in_use = (int64_t)sv->pool.used();
  return LFC_OK;
}

extern "C" lfc_status lfc_server_destroy(lfc_server *sv) {
  if (!sv) return LFC_OK;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->cv_engine.notify_all();
  if (sv->engine.joinable()) sv->engine.join();
  for (Lane &ln : sv->lanes) {
    if (ln.stream) (void)hipStreamSynchronize(ln.stream);
    if (ln.batch) (void)lfc_batch_destroy(ln.batch);
    if (ln.done) (void)hipEventDestroy(ln.done);
    if (ln.stream) (void)hipStreamDestroy(ln.stream);
  }
  if (sv->d_pool) (void)hipFree(sv->d_pool);
  delete sv;
  return LFC_OK;
}

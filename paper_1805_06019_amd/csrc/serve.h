// Internal interface between the batched render launcher (kernels.hip) and
// the batching and serving runtime (serve.cpp).  A render request is packed
// into an opaque record of render_req_bytes() bytes on the host, copied to
// the device with the others of its batch, and rendered by one launch per
// block size.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/lfc.h"

namespace lfc {

size_t render_req_bytes();

// LFC_OK if p is device memory holding at least `need` bytes (within one
// allocation) at the given alignment; else LFC_E_INVALID naming who and what.
lfc_status device_buffer(const void *p, size_t need, size_t align, const char *who, const char *what);
// Stream-ordered device scratch from the library's pool (freed with hipFreeAsync
// on the same stream); LFC_E_NOMEM if it cannot be had.
lfc_status scratch_alloc(void **p, size_t bytes, hipStream_t s);

// Packs request (view v of lf at wo x ho into out, [3][ho][wo] floats) into
// dst; reports the light field's block size, the request's tile count and
// the LDS bytes its tiles need.
lfc_status render_req_fill(const lfc_lf *lf, const lfc_view &v, int wo, int ho, float *out, void *dst, int *block,
                           int *ntiles, size_t *lds);

// One launch over n packed requests already in device memory (all of block
// size `block`): max_tiles workgroups per request, lds bytes each.
lfc_status render_multi_launch(int block, const void *d_reqs, int n, int max_tiles, size_t lds, hipStream_t s);

// The device a light field was opened on, and its block size.
int lf_device(const lfc_lf *lf);
int lf_block(const lfc_lf *lf);

// A light field's device tables for random access, packed into lf_table_bytes()
// bytes, and one launch decoding n (light field, view, block) requests of
// light fields of block size `block` whose packed tables are at d_lfs.
size_t lf_table_bytes();
void lf_table_fill(const lfc_lf *lf, void *dst);
lfc_status decode_multi_launch(int block, const void *d_lfs, int n_lf, const int32_t *d_req, int64_t n, int16_t *out,
                               int32_t *err, hipStream_t s);

// The colour decode-then-interpolate path of a batch.  A light field whose
// requests in the batch cover about as many pixels as it holds (and whose
// decoded views take less than 4 GiB) is decoded once, only the views the
// batch reads, by one persistent launch over every such light field of a
// block size (rgb_multi_launch, work items of lf_rgb_items() each, args
// packed by rgb_args_fill, counters d_ctr[2] zero before and after), into
// a scratch of lf_rgb_bytes(); then one launch interpolates every such
// request (interp_multi_launch over records packed by interp_req_fill).
bool lf_rgb_batchable(const lfc_lf *lf, double out_pixels);
size_t lf_rgb_bytes(const lfc_lf *lf);
int lf_rgb_items(const lfc_lf *lf);
int lf_views(const lfc_lf *lf);
size_t rgb_args_bytes();
void rgb_args_fill(const lfc_lf *lf, bool keys, uint32_t *d_rgb, const uint32_t *d_mask, void *dst);
size_t rgb_lds_bytes(const lfc_lf *lf, bool keys);
bool rgb_keys_fit(const lfc_lf *lf);
void need_mask_host(const lfc_lf *lf, const lfc_view &v, uint32_t *mask);
size_t interp_req_bytes();
void interp_req_fill(const lfc_lf *lf, const uint32_t *d_rgb, const lfc_view &v, int wo, int ho, float *out,
                     void *dst);
lfc_status rgb_multi_launch(int block, bool keys, const void *d_args, const int32_t *d_first, int n_lf, int n_items,
                            size_t lds, uint32_t *d_ctr, hipStream_t s);
lfc_status interp_multi_launch(const void *d_reqs, int n, int max_wo, int max_ho, hipStream_t s);

}  // namespace lfc

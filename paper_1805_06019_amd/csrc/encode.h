// Pieces of the encoder shared by the host encoder (host.cpp) and the GPU
// encoder (encode_gpu.hip), so that both write the same stream.
#pragma once

#include <cstdint>
#include <vector>

#include "internal.h"

namespace lfc {

// The 128-byte stream header (geometry, parameters, section offsets).
void put_stream_header(uint8_t *h, const Geometry &g, const lfc_params &p, uint32_t mask, uint64_t rkv_off,
                       uint64_t off_off, uint64_t srv_off);

// PSNR statistics (eq. 5 per view and channel, eq. 4, means over views) from
// the squared error of every (view, channel) on the unpadded area.
void encode_stats_from_sse(const std::vector<double> &se, int nv, int W, int H, lfc_encode_stats *stats);

}  // namespace lfc

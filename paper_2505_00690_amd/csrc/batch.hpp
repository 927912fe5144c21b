// Records a packed batch hands to the kernels through device memory.  Plain
// C++ (no device code), shared by the kernels and the host-side planner.
#pragma once

#include <stdint.h>

namespace vl {

// Per-image descriptor of a packed batch (uploaded once per call).
struct ImgDesc {
  int64_t pix_off;  // offset (floats) of the image in the pixel buffer
  int32_t H, W;     // pixel size
  int32_t gh, gw;   // patch grid
  int32_t tok_start, ntok;  // first token row in the packed stream, 1+gh*gw
};
static_assert(sizeof(ImgDesc) == 32, "ImgDesc layout");

// One attention work item: a block of up to 128 queries of one image.
struct AttnItem {
  int32_t img;
  int32_t q0;
};

// The live counts of one part of a batch, in device memory.  A launch
// sequence captured once for a capacity bucket sizes its grids for the
// capacities and passes a pointer to this record: each kernel reads the
// counts of the call being replayed and its workgroups past them return at
// once.  Launches outside such a sequence pass NULL.
struct BatchCounts {
  int32_t T;        // token rows
  int32_t n;        // images
  int32_t n_items;  // streamed attention work items
  int32_t n_res;    // K/V-resident attention images
  const float* pix; // the batch's pixel buffer (ImgDesc::pix_off is relative to it)
  float* emb;       // this part's first output row
};
static_assert(sizeof(BatchCounts) == 32, "BatchCounts layout");

}  // namespace vl

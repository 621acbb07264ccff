// Launch interface between the host runtime and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "common.h"

namespace cm {

// Device pointers of the SoA group records (see cm_groups).
struct OutPtrs {
  float *p, *n, *d, *q, *W, *logZ;
};

struct FwdArgs {
  const Entry* ents;
  int64_t n_ent;
  const QueryDev* Q;
  const ObjDesc* objs;
  DevParams P;
  uint64_t* bits;
  int32_t* nsurv;
  int32_t* ntiles;
  F4* filt;
  int64_t* bsum;
  int64_t* tile_off;
  uint32_t* counter;
  float* partials;
  const I2* gent;       // per group: (vertex entry, edge entry)
  int64_t G;
  OutPtrs out;
  float* dbg;           // nullable
  int64_t C;
  int32_t n_cu;
  int32_t blocks_per_cu;
};

hipError_t launch_grid_build(const ObjDesc* objs, const int32_t* ids, int32_t n_ids, int32_t grid_res,
                             const DevParams& P, hipStream_t s);
hipError_t launch_forward(const FwdArgs& a, hipStream_t s);

}  // namespace cm

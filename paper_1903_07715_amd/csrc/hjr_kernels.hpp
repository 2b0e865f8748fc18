// hjr_kernels.hpp -- launch wrappers of the HJI VI kernels (host side).
#pragma once

#include "hjr_device.hpp"

namespace hjr {

hipError_t launch_stage(bool fp64, const Inst *insts, const Tile *tiles, int ntiles, int stage,
                        int max_blocks, hipStream_t s);
// ev0/ev1 (optional): events stamped with the kernel's own start and end
hipError_t launch_stage_one(bool fp64, int dyn, int spatial, int npt, const Inst *insts, const Tile *tiles, int ntiles,
                            int stage, int max_blocks, hipStream_t s, hipEvent_t ev0 = nullptr,
                            hipEvent_t ev1 = nullptr, bool local = false);
hipError_t launch_step_end(const Inst *insts, int ninst, hipStream_t s);
hipError_t launch_interval(bool fp64, const Inst *insts, const Tile *tiles, int ntiles, int max_blocks,
                           hipStream_t s);
hipError_t launch_interval_end(const Inst *insts, int ninst, hipStream_t s);
// fp32_ulps: 0 = the solve starts in FP64; > 0 = it starts in FP32 with a default threshold of
// that many FP32 spacings at max |l|
hipError_t launch_init(const Inst *insts, int inst, uint32_t npts, const double *l64, const double *k64,
                       int fp32_ulps, hipStream_t s);
hipError_t launch_polish(const Inst *insts, int inst, uint32_t npts, int parity32, double shift_req,
                         hipStream_t s);
hipError_t launch_output(const Inst *insts, int inst, uint32_t npts, bool from32, int parity, double *out,
                         hipStream_t s);

}  // namespace hjr

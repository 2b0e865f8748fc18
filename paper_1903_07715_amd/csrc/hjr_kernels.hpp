// hjr_kernels.hpp -- launch wrappers of the HJI VI kernels (host side).
#pragma once

#include <vector>

#include "hjr_device.hpp"

namespace hjr {

hipError_t launch_stage(bool fp64, const Inst *insts, const Tile *tiles, int ntiles, int stage,
                        int max_blocks, hipStream_t s);
// ev0/ev1 (optional): events stamped with the kernel's own start and end
hipError_t launch_stage_one(bool fp64, int dyn, int spatial, int npt, const Inst *insts, const Tile *tiles, int ntiles,
                            int stage, int max_blocks, hipStream_t s, hipEvent_t ev0 = nullptr,
                            hipEvent_t ev1 = nullptr, bool local = false);
// Stages by the plane-march kernels (first-order upwind, or WENO5 with each dim-0 interface
// computed once): one thread per column, advancing through the dim-0 planes of its tile; one
// workgroup per tile in list order (see march_tiles for the order).  Every field of the
// instances must be below 4 GiB.  brick: the brick variant (6-D model, upwind, tiles from
// march_brick_tiles; hipErrorInvalidValue for any other model or scheme).
hipError_t launch_march(bool fp64, int dyn, int spatial, bool brick, const Inst *insts, const MTile *tiles,
                        int ntiles, int stage, hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

// The march tiles of one instance (grid dims n[0..ndim), its index `inst`), in the order its
// workgroups should run: columns are cut into tiles of at most kBlock consecutive columns within
// a row of the innermost dims, tiles are grouped into blocks of neighbouring rows (several
// dim-1 and dim-2 indices) and neighbouring tiles, and the blocks are interleaved so that
// workgroup b, which runs on XCD b mod 8, belongs to block 8 s + (b mod 8) of round s; padding
// tiles (cn = 0) keep that correspondence.  len: planes per tile (0: the whole dim-0 line).
void march_tiles(int inst, int ndim, const int *n, int len, std::vector<MTile> &out);
// The brick tiles of one 6-D instance (nothing for other ranks): a brick is rows 2k, 2k+1 of
// each of dims 1..3 and a segment of up to 128 consecutive columns of those rows (dims 4..5),
// over the whole dim-0 line; c0 is the brick's first column, cn the segment's length.  Blocks of
// neighbouring bricks are interleaved over the XCDs as in march_tiles.  The brick kernel needs
// every periodic dim among dims 1..3 to have an even number of nodes.
void march_brick_tiles(int inst, int ndim, const int *n, std::vector<MTile> &out);
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

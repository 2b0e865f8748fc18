// Safe-control queries on a resident value function (Sec. II-B.2, eq. (uOpt)): launch wrappers.
#pragma once

#include <hip/hip_runtime.h>

#include "hjr_device.hpp"

namespace hjr {

// Grid geometry of a query launch (passed by value).
struct CtlGrid {
    int ndim;
    uint32_t npts;
    uint32_t periodic;
    int n[kMaxDim];
    uint32_t stride[kMaxDim];
    double lo[kMaxDim];
    double dx[kMaxDim];
};

// Model of a query launch: game (0 avoid, 1 reach) and the model's parameters as given.
struct CtlModel {
    int game;
    double q[16];
};

// Query table: table[node * (ndim + 1) + d] = (D-_d V + D+_d V) / 2 for d < ndim with the
// solver's one-sided derivatives (spatial 1 upwind, 5 WENO5), and table[node * (ndim + 1) + ndim]
// = V at the node.
hipError_t launch_gradient(const Inst &I, int spatial, const double *V, double *table, hipStream_t s);

// Interpolated gradient, value and optimal control for nq states.
hipError_t launch_control(const CtlGrid &G, const CtlModel &M, int dyn, const double *table, const double *x,
                          int64_t nq, double *u, double *p, double *v, hipStream_t s);

}  // namespace hjr

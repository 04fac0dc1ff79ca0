// ww_batch.h -- internal types of the batched (many-patch) stage.
#pragma once
#include "ww_internal.h"

namespace ww {

// One patch of the arena: its geometry (element indices relative to the
// patch's own padded block), its three face boxes, where its padded state
// starts in the arena, and whether its x sweep uses the flattened tile.
struct PatchDesc {
    Geom G;
    FaceBox F[3];
    long soff;
    int xflat;
    int pad_;
};

template <typename T>
struct BatchArgs {
    const PatchDesc *pd;
    const int *order;          // patches by decreasing cost
    int npatch;
    int32_t *counter;          // next position in order (cleared before the stage)
    const T *u0;               // arena of the step's initial state
    T *us;                     // arena of the stage input (ghosts filled here)
    T *acc;                    // arena of the RK accumulator
    T *out;                    // arena of the stage output
    T *scratch;                // face fluxes, slot_elems per block
    long slot_elems;
    double *dt;                // per-patch time step (written in stage 0)
    int32_t *flag;             // per-patch count of non-physical cells
    double cfl;
    int s;                     // RK stage 0..3
    double bw, cw;             // weights of dt L in acc and in out
    Phys P;
};

bool batch_xflat_ok(int nx, long nrows);

template <typename T>
hipError_t launch_batch_stage(const BatchArgs<T> &a, int ft, int nblocks, hipStream_t st);

template <typename T>
hipError_t batch_occupancy(int ft, int *blocks_per_cu);

// Clear the n per-stage work counters of a step (a kernel, so that it can be
// captured in a graph).
hipError_t launch_batch_reset(int32_t *counters, int n, hipStream_t st);

}  // namespace ww

// ww_router.h -- internal declarations of the learned troubled-interface router.
#pragma once
#include "ww_internal.h"

namespace ww {

constexpr int NIN = 48, NH = 32;
constexpr int NPARAM = NH * NIN + NH + NH * NH + NH + NH + 1;   // 2657

hipError_t launch_mlp_infer(const float *th, const float *X, int n, float *logit, hipStream_t st);
int mlp_grad_blocks(int n);
hipError_t launch_mlp_grad(const float *th, const float *X, const float *t, int n, float *part,
                           float *grad, float *loss, hipStream_t st);
hipError_t launch_mlp_adam(float *th, float *m, float *v, const float *grad, int step, float lr,
                           float b1, float b2, float eps, hipStream_t st);
template <typename T>
hipError_t launch_router_sample(const T *u, const Geom &G, const Phys &P, const int32_t *where,
                                int n, float *X, float *dev, float *ex, hipStream_t st);
constexpr int MLP_PACKED_BYTES = 10 * 64 * 8 + 25 * 64 * 4;
hipError_t launch_pack_mlp(const float *th, char *pk, hipStream_t st);
long routed_sweep_blocks(int dir, const FaceBox &F);
// Troubled-queue entries the routed sweep of direction dir may need: 64
// regions of ceil(blocks / 64) * 256 entries; qcount holds 64 counters.
long routed_queue_capacity(int dir, const FaceBox &F);
constexpr int ROUTED_QUEUE_REGIONS = 64;
// Routed sweep of direction dir (force 0 routed, -1 all linear), then the
// full-WENO pass over the queued troubled interfaces.  queue holds
// 64 * routed_queue_capacity(dir, F) entries; the 64 counters in qcount are
// cleared on st first.  mask (F.sc bytes) receives
// the decisions, or supplies them when reuse is set.  xf (x sweep of a 3-D
// box with rows of at least sweep_x_fused_min_faces() faces, after the y and
// z sweeps; else nullptr): also the rho, m, E part of the RK stage, as the
// fused x sweep does; the update then does B only.
hipError_t launch_routed_sweep(int dir, const float *u, float *flux, const Geom &G, const FaceBox &F,
                              const Phys &P, const char *pk, float thr, int force, int32_t *nsmooth,
                              unsigned long long *queue, int32_t *qcount, unsigned char *mask, int reuse,
                              const XFuse<float> *xf, hipStream_t st);

}  // namespace ww

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
long learned_sweep_blocks(int dir, const FaceBox &F);
hipError_t launch_learned_sweep(int dir, const float *u, float *flux, const Geom &G, const FaceBox &F,
                                const Phys &P, const float *th, float thr, int force,
                                int32_t *nsmooth, hipStream_t st);

}  // namespace ww

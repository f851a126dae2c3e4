// Launchers of the single-mesh SSD kernels (device bodies in ssd_tiles.h).
#include <hip/hip_ext.h>

#include "ssd_launch.h"
#include "ssd_tiles.h"

namespace ssd {

hipError_t launch_traces(const DevMesh &M, const OpTables &T, const float *q, float *tr,
                         hipStream_t s) {
  const int grid = (M.E + TRACE_BLOCK - 1) / TRACE_BLOCK;
  SSD_DISPATCH_N(M.N, hipLaunchKernelGGL(k_traces<NN>, dim3(grid), dim3(TRACE_BLOCK), 0, s, M, T,
                                         q, tr));
  return hipGetLastError();
}

hipError_t launch_rebuild(const DevMesh &M, const MortarTables &MT, double theta, MortarState *ms,
                          hipStream_t s) {
  SSD_DISPATCH_N(M.N, hipLaunchKernelGGL(k_rebuild<NN>, dim3(1), dim3(64), 0, s, M, MT, theta,
                                         ms));
  return hipGetLastError();
}

hipError_t launch_mortar(const DevMesh &M, const OpTables &T, const MortarTables &MT,
                         double theta, MortarState *ms, const float *tr, float *mflux, float *mqc,
                         hipStream_t s) {
  SSD_DISPATCH_N(M.N, {
    const int grid = (2 * M.K + MORTAR_BLOCK / NN - 1) / (MORTAR_BLOCK / NN);
    if (mqc)
      hipLaunchKernelGGL((k_mortar<NN, true>), dim3(grid), dim3(MORTAR_BLOCK), 0, s, M, T, MT,
                         theta, ms, tr, mflux, mqc);
    else
      hipLaunchKernelGGL((k_mortar<NN, false>), dim3(grid), dim3(MORTAR_BLOCK), 0, s, M, T, MT,
                         theta, ms, tr, mflux, mqc);
  });
  return hipGetLastError();
}

hipError_t launch_mortar_visc(const DevMesh &M, const OpTables &T, const MortarState *ms,
                              const float *mqc, const float *gtr, float *mvflux, hipStream_t s) {
  SSD_DISPATCH_N(M.N, {
    const int grid = (2 * M.K + MORTAR_BLOCK / NN - 1) / (MORTAR_BLOCK / NN);
    hipLaunchKernelGGL(k_mortar_visc<NN>, dim3(grid), dim3(MORTAR_BLOCK), 0, s, M, T, ms, mqc,
                       gtr, mvflux);
  });
  return hipGetLastError();
}

hipError_t launch_grad(const DevMesh &M, const OpTables &T, Rotation rot, const float *q,
                       const float *facein, float *G, float *gtr, hipStream_t s, bool reverse) {
  const int grid = (M.E + EB - 1) / EB;
  SSD_DISPATCH_N(M.N, hipLaunchKernelGGL(k_grad<NN>, dim3(grid), dim3(EB * NN), 0, s, M, T, rot, q,
                                         facein, G, gtr, int(reverse)));
  return hipGetLastError();
}

hipError_t launch_stage(const DevMesh &M, const OpTables &T, Rotation rot, const float *q,
                        const float *qn, float *out, const float *facein, float *trout,
                        const ViscIO *visc, const RKCoef &C, bool rk, hipStream_t s,
                        hipEvent_t ev0, hipEvent_t ev1) {
  const int grid = (M.E + EB - 1) / EB;
  const ViscBufs V{visc ? visc->G : nullptr, visc ? visc->gtr : nullptr,
                   visc ? visc->mvflux : nullptr};
#define SSD_STAGE(RKV, VV, AV, CV)                                                           \
  SSD_DISPATCH_N(M.N, hipExtLaunchKernelGGL((k_stage<NN, RKV, VV, AV, CV>), dim3(grid),         \
                                            dim3(EB * NN), 0, s, ev0, ev1, 0, M, T, rot, q, qn, out, \
                                            facein, trout, V, C))
  const bool add = rk && C.add != nullptr;
  if (rk && C.comb) {   // SSPRK54 fourth stage with the increment (never with add)
    if (add || !qn) return hipErrorInvalidValue;
    if (visc) {
      SSD_STAGE(true, true, false, true);
    } else {
      SSD_STAGE(true, false, false, true);
    }
  } else if (rk && visc) {
    if (add) {
      SSD_STAGE(true, true, true, false);
    } else {
      SSD_STAGE(true, true, false, false);
    }
  } else if (rk) {
    if (add) {
      SSD_STAGE(true, false, true, false);
    } else {
      SSD_STAGE(true, false, false, false);
    }
  } else if (visc) {
    SSD_STAGE(false, true, false, false);
  } else {
    SSD_STAGE(false, false, false, false);
  }
#undef SSD_STAGE
  return hipGetLastError();
}

}  // namespace ssd

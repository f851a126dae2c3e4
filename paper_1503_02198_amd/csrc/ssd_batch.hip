// Batched execution of many meshes: the tile and chunk bodies of
// ssd_tiles.h driven by device tables of (case, tile or chunk) items.
#include "ssd_launch.h"
#include "ssd_tiles.h"

namespace ssd {

// ---------------------------------------------------------------------------
// batched kernels: the tile and chunk bodies over a table of
// (case, tile or chunk) items, one item per block.  A persistent grid-stride
// loop over the items was measured slower: the compiler hoists per-tile
// values out of the loop and the stage kernel loses half its occupancy.
// ---------------------------------------------------------------------------
// Rotation of a case at stage time offset c of step *step.
__device__ __forceinline__ Rotation batch_rotation(const BatchCase &B, const double *step,
                                                   double c) {
  const double th = B.theta0 + B.omega * (B.t0 + (step[0] + c) * B.dt);
  double sn, cs;
  sincos(th, &sn, &cs);
  return Rotation{cs, sn, B.omega};
}

__device__ __forceinline__ uint2 batch_item(const uint2 *work, bool reverse = false) {
  const uint2 w = work[reverse ? gridDim.x - 1 - blockIdx.x : blockIdx.x];
  return make_uint2(__builtin_amdgcn_readfirstlane(w.x), __builtin_amdgcn_readfirstlane(w.y));
}

template <int N>
__global__ __launch_bounds__(TRACE_BLOCK) void kb_traces(const BatchCase *cases, const uint2 *work,
                                                         OpTables T) {
  const uint2 it = batch_item(work);
  const BatchCase &B = cases[it.x];
  traces_block<N>(B.M, T, B.buf[0], B.face[0], int(it.y));
}

template <int N, bool VISC>
__global__ __launch_bounds__(MORTAR_BLOCK) void kb_mortar(const BatchCase *cases, const uint2 *work,
                                                          OpTables T, MortarTables MT, int cur,
                                                          double c, const double *step) {
  const uint2 it = batch_item(work);
  const BatchCase &B = cases[it.x];
  const double theta = B.theta0 + B.omega * (B.t0 + (step[0] + c) * B.dt);
  float *fb = B.face[cur];
  const long nt = 16L * N * B.M.E, nr = 8L * B.M.K * N;
  mortar_chunk<N, VISC>(B.M, T, MT, theta, B.ms, fb, fb + nt, VISC ? fb + nt + nr : nullptr,
                        int(it.y));
}

template <int N>
__global__ __launch_bounds__(64 * N) void kb_grad(const BatchCase *cases, const uint2 *work,
                                                  OpTables T, int in, int cur, double c,
                                                  const double *step) {
  const uint2 it = batch_item(work);
  const BatchCase &B = cases[it.x];
  const Rotation R = batch_rotation(B, step, c);
  grad_tile<N>(B.M, T, R, B.buf[in], B.face[cur], B.V.G, B.V.gtr, int(it.y));
}

template <int N>
__global__ __launch_bounds__(MORTAR_BLOCK) void kb_mortar_visc(const BatchCase *cases,
                                                               const uint2 *work, OpTables T,
                                                               int cur) {
  const uint2 it = batch_item(work);
  const BatchCase &B = cases[it.x];
  const float *fb = B.face[cur];
  const long nt = 16L * N * B.M.E, nr = 8L * B.M.K * N;
  mortar_visc_chunk<N>(B.M, T, B.ms, fb + nt + nr, B.V.gtr, B.V.mvflux, int(it.y));
}

// TPB consecutive items of the work table per block (the tile shape the
// autotuner picks per group); groups of N waves each, see stage_tile.
template <int N, bool VISC, bool ADD, bool COMB = false, int TPB = 1>
__global__ __launch_bounds__(64 * N * TPB)
__attribute__((amdgpu_waves_per_eu(stage_waves_per_eu<N, true, VISC, ADD, COMB>()))) void kb_stage(
    const BatchCase *cases, const uint2 *work, int nwork, OpTables T, BatchStage S,
    const double *step) {
  const int b = S.reverse ? int(gridDim.x) - 1 - int(blockIdx.x) : int(blockIdx.x);
  const int grp = TPB > 1 ? __builtin_amdgcn_readfirstlane(int(threadIdx.x) / (64 * N)) : 0;
  const int idx = b * TPB + grp;
  const bool active = idx < nwork;
  const uint2 w = work[active ? idx : b * TPB];
  const uint2 it = make_uint2(__builtin_amdgcn_readfirstlane(w.x), __builtin_amdgcn_readfirstlane(w.y));
  const BatchCase &B = cases[it.x];
  const Rotation R = batch_rotation(B, step, S.c);
  const ViscBufs V{B.V.G, B.V.gtr, B.V.mvflux};
  RKCoef C{S.beta, S.gamma, float(B.dt), ADD ? B.buf[S.add] : nullptr};
  if (COMB) {
    C.comb = B.buf[S.comb];
    C.cw2 = S.cw2;
    C.cw3 = S.cw3;
    C.cw4 = S.cw4;
  }
  stage_tile<N, true, VISC, ADD, COMB, TPB>(B.M, T, R, B.buf[S.in],
                                            S.qn >= 0 ? B.buf[S.qn] : nullptr, B.buf[S.out],
                                            B.face[S.cur], B.face[S.cur ^ 1], V, C, int(it.y),
                                            active);
}

__global__ void k_step_count(double *step) {
  if (threadIdx.x == 0) step[0] += 1.0;
}

hipError_t launch_batch_traces(int N, const BatchCase *cases, const uint2 *work, int nwork,
                               const OpTables &T, hipStream_t s) {
  if (nwork < 1) return hipSuccess;
  SSD_DISPATCH_N(N, hipLaunchKernelGGL(kb_traces<NN>, dim3(nwork), dim3(TRACE_BLOCK), 0, s, cases,
                                       work, T));
  return hipGetLastError();
}

hipError_t launch_batch_mortar(int N, bool visc, const BatchCase *cases, const uint2 *work,
                               int nwork, const OpTables &T, const MortarTables &MT, int cur,
                               double c, const double *step, hipStream_t s) {
  if (nwork < 1) return hipSuccess;
  if (visc) {
    SSD_DISPATCH_N(N, hipLaunchKernelGGL((kb_mortar<NN, true>), dim3(nwork), dim3(MORTAR_BLOCK),
                                         0, s, cases, work, T, MT, cur, c, step));
  } else {
    SSD_DISPATCH_N(N, hipLaunchKernelGGL((kb_mortar<NN, false>), dim3(nwork), dim3(MORTAR_BLOCK),
                                         0, s, cases, work, T, MT, cur, c, step));
  }
  return hipGetLastError();
}

hipError_t launch_batch_grad(int N, const BatchCase *cases, const uint2 *work, int nwork,
                             const OpTables &T, int in, int cur, double c, const double *step,
                             hipStream_t s) {
  if (nwork < 1) return hipSuccess;
  SSD_DISPATCH_N(N, hipLaunchKernelGGL(kb_grad<NN>, dim3(nwork), dim3(EB * NN), 0, s, cases, work,
                                       T, in, cur, c, step));
  return hipGetLastError();
}

hipError_t launch_batch_mortar_visc(int N, const BatchCase *cases, const uint2 *work, int nwork,
                                    const OpTables &T, int cur, hipStream_t s) {
  if (nwork < 1) return hipSuccess;
  SSD_DISPATCH_N(N, hipLaunchKernelGGL(kb_mortar_visc<NN>, dim3(nwork), dim3(MORTAR_BLOCK), 0, s,
                                       cases, work, T, cur));
  return hipGetLastError();
}

hipError_t launch_batch_stage(int N, bool visc, const BatchCase *cases, const uint2 *work,
                              int nwork, const OpTables &T, const BatchStage &S,
                              const double *step, hipStream_t s, int tpb) {
  if (nwork < 1) return hipSuccess;
  if (tpb != 1 && !(tpb == 2 && N <= 4)) return hipErrorInvalidValue;
  const int nblk = (nwork + tpb - 1) / tpb;
#define SSD_BSTAGE(VV, AV, CV)                                                                 \
  do {                                                                                         \
    if (tpb == 1) {                                                                            \
      SSD_DISPATCH_N(N, hipLaunchKernelGGL((kb_stage<NN, VV, AV, CV, 1>), dim3(nblk),          \
                                           dim3(EB * NN), 0, s, cases, work, nwork, T, S, step)); \
    } else {                                                                                   \
      SSD_DISPATCH_N_SMALL(N, hipLaunchKernelGGL((kb_stage<NN, VV, AV, CV, 2>), dim3(nblk),    \
                                           dim3(2 * EB * NN), 0, s, cases, work, nwork, T, S,   \
                                           step));                                             \
    }                                                                                          \
  } while (0)
  const bool add = S.add >= 0;
  if (S.comb >= 0) {   // SSPRK54's fourth stage with the increment (never with add)
    if (add || S.qn < 0) return hipErrorInvalidValue;
    if (visc) {
      SSD_BSTAGE(true, false, true);
    } else {
      SSD_BSTAGE(false, false, true);
    }
  } else if (visc) {
    if (add) {
      SSD_BSTAGE(true, true, false);
    } else {
      SSD_BSTAGE(true, false, false);
    }
  } else {
    if (add) {
      SSD_BSTAGE(false, true, false);
    } else {
      SSD_BSTAGE(false, false, false);
    }
  }
#undef SSD_BSTAGE
  return hipGetLastError();
}

hipError_t launch_step_count(double *step, hipStream_t s) {
  hipLaunchKernelGGL(k_step_count, dim3(1), dim3(64), 0, s, step);
  return hipGetLastError();
}

}  // namespace ssd

// Measurement probe behind a design decision of the stage kernel: the
// per-cell contractions of the flux-point method (Sec. 3.1 eqs. Qt, Ft, Gt:
// interpolation I from the N solution points of a line to its N + 1 flux
// points, a pointwise flux, the derivative D back to the solution points),
// done two ways over the stage kernel's data layout (lane = cell, wave =
// line, 64 cells per wave):
//   variant 0  VALU: each lane runs the (N+1) x N and N x (N+1) products of
//              its own cell with fused multiply-adds, as the stage kernel does;
//   variant 1  MFMA: v_mfma_f32_16x16x4_f32 with the operator as the A
//              matrix (flux points, or solution points, as rows, padded to
//              16) and 16 cells as the columns of B; the lane = cell rows
//              are moved into the B layout, and the results back, through
//              LDS.
// The pointwise flux is f = q^2 (nonlinear, so that the two products do not
// collapse into one), and the line takes `reps` explicit steps
// q <- q - 0.01 D f(I q) in registers (Burgers' equation along the line;
// the values stay of order one), so that the arithmetic, not the 8 bytes per
// point of memory traffic, sets the time.  N = 4.
//
// A second probe measures the bandwidth ceiling of the stage kernel's state
// traffic: c = 0.75 a + 0.25 b, two arrays read and one written, as an
// SSP-RK stage reads Q and Qn and writes the new state (see
// launch_stream_probe for the access variants).
#include <hip/hip_runtime.h>

#include "ssd_device.h"
#include "ssd_launch.h"

namespace ssd {
namespace {

constexpr int PN = 4;   // solution points per line

typedef float f32x4 __attribute__((ext_vector_type(4)));

struct ProbeOps {
  float I[PN + 1][PN];   // solution points -> flux points
  float D[PN][PN + 1];   // flux points -> derivative at solution points, times -0.01
};

// variant 0: lane = cell; q, out [4][PN lines][PN points][E] (cell fastest)
__global__ __launch_bounds__(64 * PN) void k_probe_valu(ProbeOps P, const float *q, float *out,
                                                          int E, int reps) {
  const int w = __builtin_amdgcn_readfirstlane(int(threadIdx.x) / 64);
  const int cell = int(blockIdx.x) * 64 + int(threadIdx.x & 63);
  if (cell >= E) return;
  float x[4][PN];
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int i = 0; i < PN; ++i) x[v][i] = q[size_t((v * PN + w) * PN + i) * E + cell];
  for (int r = 0; r < reps; ++r) {
    float res[4][PN];
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int i = 0; i < PN; ++i) res[v][i] = x[v][i];
#pragma unroll
    for (int k = 0; k <= PN; ++k) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        float a = 0.f;
#pragma unroll
        for (int i = 0; i < PN; ++i) a += P.I[k][i] * x[v][i];
        const float f = a * a;
#pragma unroll
        for (int i = 0; i < PN; ++i) res[v][i] += P.D[i][k] * f;
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int i = 0; i < PN; ++i) x[v][i] = res[v][i];
  }
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int i = 0; i < PN; ++i) out[size_t((v * PN + w) * PN + i) * E + cell] = x[v][i];
}

// variant 1: the same arithmetic on the matrix cores.  v_mfma_f32_16x16x4_f32
// takes A[m][k] from lane m + 16 k, B[k][n] from lane n + 16 k, and leaves
// D[m][n] in register m % 4 of lane n + 16 (m / 4).  Each wave moves its
// rows between the lane = cell layout and those layouts through its own
// LDS area (no other wave touches it, so no barrier is needed).
__global__ __launch_bounds__(64 * PN) void k_probe_mfma(ProbeOps P, const float *q, float *out,
                                                          int E, int reps) {
  __shared__ float Lx[PN][PN][64];       // [wave][solution point][cell]
  __shared__ float Lm[PN][16][17];       // [wave][matrix row][column], padded
  const int w = __builtin_amdgcn_readfirstlane(int(threadIdx.x) / 64);
  const int lane = int(threadIdx.x & 63);
  const int cell = int(blockIdx.x) * 64 + lane;
  const bool ok = cell < E;   // E is a multiple of 64 (checked on the host)
  // A operands: the interpolation (flux-point rows, K = solution points)
  // and the two K = 4 halves of the derivative (solution-point rows, K =
  // flux points 0..3 and 4..7); rows and columns past the operators are 0
  const int m = lane & 15, kk = lane >> 4;
  const float aI = m <= PN ? P.I[m][kk] : 0.f;
  const float aD0 = m < PN ? P.D[m][kk] : 0.f;
  const float aD1 = (m < PN && 4 + kk <= PN) ? P.D[m][4 + kk] : 0.f;
  float x[4][PN];
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int i = 0; i < PN; ++i) x[v][i] = ok ? q[size_t((v * PN + w) * PN + i) * E + cell] : 0.f;
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
  for (int r = 0; r < reps; ++r) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
#pragma unroll
      for (int i = 0; i < PN; ++i) Lx[w][i][lane] = x[v][i];
      float nx[PN];
#pragma unroll
      for (int g = 0; g < 4; ++g) {   // 16-cell groups
        // B: solution point kk of cell 16 g + m
        const f32x4 F = __builtin_amdgcn_mfma_f32_16x16x4f32(aI, Lx[w][kk][16 * g + m], zero, 0,
                                                              0, 0);
        // F[flux point][cell] squared, to LDS, then the two B halves
#pragma unroll
        for (int t = 0; t < 4; ++t) Lm[w][4 * kk + t][m] = F[t] * F[t];
        const float b0 = Lm[w][kk][m], b1 = Lm[w][4 + kk][m];
        f32x4 R = __builtin_amdgcn_mfma_f32_16x16x4f32(aD0, b0, zero, 0, 0, 0);
        R = __builtin_amdgcn_mfma_f32_16x16x4f32(aD1, b1, R, 0, 0, 0);
        // R[solution point][cell] to LDS; the cell's lane takes its column
#pragma unroll
        for (int t = 0; t < 4; ++t) Lm[w][4 * kk + t][m] = R[t];
        if ((lane >> 4) == g) {
#pragma unroll
          for (int i = 0; i < PN; ++i) nx[i] = Lm[w][i][m];
        }
      }
#pragma unroll
      for (int i = 0; i < PN; ++i) x[v][i] += nx[i];
    }
  }
  if (!ok) return;
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int i = 0; i < PN; ++i) out[size_t((v * PN + w) * PN + i) * E + cell] = x[v][i];
}

}  // namespace
}  // namespace ssd

namespace ssd {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

// 16 bytes per lane and array; one block covers 1024 floats
template <bool NT>
__global__ __launch_bounds__(256) void k_stream_x4(const v4f *a, const v4f *b, v4f *c) {
  const size_t i = size_t(blockIdx.x) * 256 + threadIdx.x;
  v4f x, y;
  if (NT) {
    x = __builtin_nontemporal_load(a + i);
    y = __builtin_nontemporal_load(b + i);
  } else {
    x = a[i];
    y = b[i];
  }
  const v4f z = 0.75f * x + 0.25f * y;
  if (NT)
    __builtin_nontemporal_store(z, c + i);
  else
    c[i] = z;
}

// the stage kernel's access: 4-byte non-temporal buffer loads and stores per
// lane, each wave instruction covering one 256-byte row; a wave takes 4
// consecutive rows, a block 1024 floats
__global__ __launch_bounds__(256) void k_stream_rows(const float *a, const float *b, float *c,
                                                     uint32_t bytes) {
  const rsrc_t ra = make_rsrc(a, bytes), rb = make_rsrc(b, bytes), rc = make_rsrc(c, bytes);
  const uint32_t wave = uint32_t(__builtin_amdgcn_readfirstlane(int(threadIdx.x) / 64));
  const uint32_t base = (blockIdx.x * 1024u + wave * 256u) * 4u;
  const uint32_t lane = (threadIdx.x & 63u) * 4u;
  float x[4], y[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    x[k] = bload_nt(ra, lane, base + k * 256u);
    y[k] = bload_nt(rb, lane, base + k * 256u);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) bstore_nt(0.75f * x[k] + 0.25f * y[k], rc, lane, base + k * 256u);
}

}  // namespace

// n: a positive multiple of 1024 with 4 n < 2^32 (checked by the caller)
hipError_t launch_stream_probe(int variant, int64_t n, const float *a, const float *b, float *c,
                               hipStream_t s) {
  const dim3 grid(unsigned(n / 1024)), block(256);
  if (variant == 0)
    hipLaunchKernelGGL(k_stream_x4<false>, grid, block, 0, s, (const v4f *)a, (const v4f *)b,
                       (v4f *)c);
  else if (variant == 1)
    hipLaunchKernelGGL(k_stream_x4<true>, grid, block, 0, s, (const v4f *)a, (const v4f *)b,
                       (v4f *)c);
  else
    hipLaunchKernelGGL(k_stream_rows, grid, block, 0, s, a, b, c, uint32_t(n * 4));
  return hipGetLastError();
}

hipError_t launch_probe(int variant, const OpTables &T, int n_cells, int reps, const float *q,
                        float *out, hipStream_t s) {
  ProbeOps P;
  for (int k = 0; k <= PN; ++k)
    for (int i = 0; i < PN; ++i) {
      P.I[k][i] = T.I[k][i];
      P.D[i][k] = -0.01f * T.D[i][k];
    }
  const dim3 grid(n_cells / 64), block(64 * PN);
  if (variant == 0)
    hipLaunchKernelGGL(k_probe_valu, grid, block, 0, s, P, q, out, n_cells, reps);
  else
    hipLaunchKernelGGL(k_probe_mfma, grid, block, 0, s, P, q, out, n_cells, reps);
  return hipGetLastError();
}

}  // namespace ssd

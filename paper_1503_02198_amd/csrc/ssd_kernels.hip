// HIP kernels of the SSD residual for gfx950 (CDNA4).
//
// Layout: SoA with the element index fastest.  One lane owns one element:
// its N x N x 4 state sits in VGPRs, so every global access of a wave is a
// contiguous 256-byte row per (variable, point).  Face traces (the solution
// interpolated to the element-boundary flux points) travel between
// neighbours through a trace buffer [face][point][var][E]; the neighbour
// read is a gather that is contiguous whenever consecutive elements have
// consecutive neighbours (structured O-grids numbered azimuth-fastest).
//
// Precision: state, traces and fluxes in FP32; element metrics and the
// sliding-interface projections in FP64.
#include "ssd_internal.h"

namespace ssd {

// ---------------------------------------------------------------------------
// fluxes (Sec. 2.1, 2.2, 3.1)
// ---------------------------------------------------------------------------
// Normal inviscid ALE flux along the scaled normal (nx, ny):
// (F - u_g Q) nx + (G - v_g Q) ny with vgn = u_g nx + v_g ny.
__device__ __forceinline__ void flux_n(const float q[4], float nx, float ny, float vgn, float gm1,
                                       float f[4]) {
  const float ir = 1.0f / q[0];
  const float u = q[1] * ir, v = q[2] * ir;
  const float p = gm1 * (q[3] - 0.5f * (q[1] * u + q[2] * v));
  const float un = u * nx + v * ny;
  const float rel = un - vgn;
  f[0] = q[0] * rel;
  f[1] = q[1] * rel + p * nx;
  f[2] = q[2] * rel + p * ny;
  f[3] = q[3] * rel + p * un;
}

// Rusanov common flux from the owner (l) towards the neighbour (r).
__device__ __forceinline__ void rusanov(const float ql[4], const float qr[4], float nx, float ny,
                                        float vgn, float gam, float f[4]) {
  const float gm1 = gam - 1.0f;
  const float mag = sqrtf(nx * nx + ny * ny);
  const float irl = 1.0f / ql[0], irr = 1.0f / qr[0];
  const float ul = ql[1] * irl, vl = ql[2] * irl;
  const float ur = qr[1] * irr, vr = qr[2] * irr;
  const float pl = gm1 * (ql[3] - 0.5f * (ql[1] * ul + ql[2] * vl));
  const float pr = gm1 * (qr[3] - 0.5f * (qr[1] * ur + qr[2] * vr));
  const float unl = ul * nx + vl * ny, unr = ur * nx + vr * ny;
  const float rl = unl - vgn, rr = unr - vgn;
  const float cl = sqrtf(gam * pl * irl), cr = sqrtf(gam * pr * irr);
  const float lam = fmaxf(fabsf(rl) + cl * mag, fabsf(rr) + cr * mag);
  f[0] = 0.5f * (ql[0] * rl + qr[0] * rr) - 0.5f * lam * (qr[0] - ql[0]);
  f[1] = 0.5f * (ql[1] * rl + pl * nx + qr[1] * rr + pr * nx) - 0.5f * lam * (qr[1] - ql[1]);
  f[2] = 0.5f * (ql[2] * rl + pl * ny + qr[2] * rr + pr * ny) - 0.5f * lam * (qr[2] - ql[2]);
  f[3] = 0.5f * (ql[3] * rl + pl * unl + qr[3] * rr + pr * unr) - 0.5f * lam * (qr[3] - ql[3]);
}

// FP64 Rusanov flux for the mortars (no grid velocity: u_g . n = 0 on the circle).
__device__ __forceinline__ void rusanov_d(const double ql[4], const double qr[4], double nx,
                                          double ny, double gam, double f[4]) {
  const double gm1 = gam - 1.0;
  const double mag = sqrt(nx * nx + ny * ny);
  const double ul = ql[1] / ql[0], vl = ql[2] / ql[0];
  const double ur = qr[1] / qr[0], vr = qr[2] / qr[0];
  const double pl = gm1 * (ql[3] - 0.5 * (ql[1] * ul + ql[2] * vl));
  const double pr = gm1 * (qr[3] - 0.5 * (qr[1] * ur + qr[2] * vr));
  const double unl = ul * nx + vl * ny, unr = ur * nx + vr * ny;
  const double cl = sqrt(gam * pl / ql[0]), cr = sqrt(gam * pr / qr[0]);
  const double lam = fmax(fabs(unl) + cl * mag, fabs(unr) + cr * mag);
  f[0] = 0.5 * (ql[0] * unl + qr[0] * unr) - 0.5 * lam * (qr[0] - ql[0]);
  f[1] = 0.5 * (ql[1] * unl + pl * nx + qr[1] * unr + pr * nx) - 0.5 * lam * (qr[1] - ql[1]);
  f[2] = 0.5 * (ql[2] * unl + pl * ny + qr[2] * unr + pr * ny) - 0.5 * lam * (qr[2] - ql[2]);
  f[3] = 0.5 * (ql[3] * unl + pl * unl + qr[3] * unr + pr * unr) - 0.5 * lam * (qr[3] - ql[3]);
}

// ---------------------------------------------------------------------------
// element geometry (Sec. 2.3): bilinear cells from their corners, cubic
// cells from precomputed FP64 tables; zone-1 cells rotated by theta.
// ---------------------------------------------------------------------------
struct ElemGeo {
  int cubic, c;
  double ct, st, w;
  double x0, y0, x3, y3, x6, y6, x9, y9;
};

__device__ __forceinline__ ElemGeo load_geo(const DevMesh &M, int e, const Rotation &R) {
  ElemGeo g;
  const int fl = M.eflag[e];
  g.cubic = fl & EF_CUBIC;
  g.c = fl >> 8;
  const bool rot = (fl & EF_ROT) != 0;
  g.ct = rot ? R.ct : 1.0;
  g.st = rot ? R.st : 0.0;
  g.w = rot ? R.omega : 0.0;
  const long E = M.E;
  if (!g.cubic) {
    g.x0 = M.corners[0 * E + e];
    g.y0 = M.corners[1 * E + e];
    g.x3 = M.corners[2 * E + e];
    g.y3 = M.corners[3 * E + e];
    g.x6 = M.corners[4 * E + e];
    g.y6 = M.corners[5 * E + e];
    g.x9 = M.corners[6 * E + e];
    g.y9 = M.corners[7 * E + e];
  } else {
    g.x0 = g.y0 = g.x3 = g.y3 = g.x6 = g.y6 = g.x9 = g.y9 = 0.0;
  }
  return g;
}

// Scaled normal (y_eta, -x_eta) of the xi-direction flux point (Xf_k, X_j)
// in the rotated frame, and u_g . n (rotation invariant, body frame).
template <int N>
__device__ __forceinline__ void metric_xi(const ElemGeo &g, const DevMesh &M, const OpTables &T,
                                          int k, int j, float &nx, float &ny, float &vgn) {
  double xe, ye, px = 0.0, py = 0.0;
  if (g.cubic) {
    xe = M.cmet[cubic_xi_index(N, M.C, 0, j, k, g.c)];
    ye = M.cmet[cubic_xi_index(N, M.C, 1, j, k, g.c)];
    if (g.w != 0.0) {
      px = M.cmet[cubic_xi_index(N, M.C, 2, j, k, g.c)];
      py = M.cmet[cubic_xi_index(N, M.C, 3, j, k, g.c)];
    }
  } else {
    const double xi = T.Xf[k], eta = T.X[j];
    xe = (1.0 - xi) * (g.x9 - g.x0) + xi * (g.x6 - g.x3);
    ye = (1.0 - xi) * (g.y9 - g.y0) + xi * (g.y6 - g.y3);
    if (g.w != 0.0) {
      const double a0 = (1.0 - xi) * (1.0 - eta), a3 = xi * (1.0 - eta), a6 = xi * eta,
                   a9 = (1.0 - xi) * eta;
      px = a0 * g.x0 + a3 * g.x3 + a6 * g.x6 + a9 * g.x9;
      py = a0 * g.y0 + a3 * g.y3 + a6 * g.y6 + a9 * g.y9;
    }
  }
  const double xr = g.ct * xe - g.st * ye;
  const double yr = g.st * xe + g.ct * ye;
  nx = float(yr);
  ny = float(-xr);
  vgn = float(-g.w * (px * xe + py * ye));
}

// Scaled normal (-y_xi, x_xi) of the eta-direction flux point (X_i, Xf_k).
template <int N>
__device__ __forceinline__ void metric_eta(const ElemGeo &g, const DevMesh &M, const OpTables &T,
                                           int k, int i, float &nx, float &ny, float &vgn) {
  double xx, yx, px = 0.0, py = 0.0;
  if (g.cubic) {
    xx = M.cmet[cubic_eta_index(N, M.C, 0, k, i, g.c)];
    yx = M.cmet[cubic_eta_index(N, M.C, 1, k, i, g.c)];
    if (g.w != 0.0) {
      px = M.cmet[cubic_eta_index(N, M.C, 2, k, i, g.c)];
      py = M.cmet[cubic_eta_index(N, M.C, 3, k, i, g.c)];
    }
  } else {
    const double xi = T.X[i], eta = T.Xf[k];
    xx = (1.0 - eta) * (g.x3 - g.x0) + eta * (g.x6 - g.x9);
    yx = (1.0 - eta) * (g.y3 - g.y0) + eta * (g.y6 - g.y9);
    if (g.w != 0.0) {
      const double a0 = (1.0 - xi) * (1.0 - eta), a3 = xi * (1.0 - eta), a6 = xi * eta,
                   a9 = (1.0 - xi) * eta;
      px = a0 * g.x0 + a3 * g.x3 + a6 * g.x6 + a9 * g.x9;
      py = a0 * g.y0 + a3 * g.y3 + a6 * g.y6 + a9 * g.y9;
    }
  }
  const double xr = g.ct * xx - g.st * yx;
  const double yr = g.st * xx + g.ct * yx;
  nx = float(-yr);
  ny = float(xr);
  vgn = float(g.w * (px * xx + py * yx));
}

template <int N>
__device__ __forceinline__ double jacobian(const ElemGeo &g, const DevMesh &M, const OpTables &T,
                                           int j, int i) {
  if (g.cubic) return M.cmet[cubic_sp_index(N, M.C, 0, j, i, g.c)];
  const double xi = T.X[i], eta = T.X[j];
  const double xx = (1.0 - eta) * (g.x3 - g.x0) + eta * (g.x6 - g.x9);
  const double yx = (1.0 - eta) * (g.y3 - g.y0) + eta * (g.y6 - g.y9);
  const double xe = (1.0 - xi) * (g.x9 - g.x0) + xi * (g.x6 - g.x3);
  const double ye = (1.0 - xi) * (g.y9 - g.y0) + xi * (g.y6 - g.y3);
  return xx * ye - xe * yx;
}

// ---------------------------------------------------------------------------
// common normal flux at one element-boundary flux point (outward normal)
// ---------------------------------------------------------------------------
template <int N>
__device__ __forceinline__ void common_flux(const DevMesh &M, uint32_t w, int p, const float qo[4],
                                            float nx, float ny, float vgn,
                                            const float *__restrict__ trin,
                                            const float *__restrict__ mflux, float fs[4]) {
  const int kind = face_kind_of(w);
  const long E = M.E;
  if (kind == SSD_FACE_INTERIOR || kind == SSD_FACE_PERIODIC) {
    const int nb = face_idx_of(w), nf = face_nf_of(w);
    const int pp = face_rev_of(w) ? N - 1 - p : p;
    float qr[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) qr[v] = trin[long((nf * N + pp) * 4 + v) * E + nb];
    rusanov(qo, qr, nx, ny, vgn, M.gamma, fs);
  } else if (kind == SSD_FACE_SLIDING) {
    const int slot = face_idx_of(w);
    const long S = 2L * M.K;
#pragma unroll
    for (int v = 0; v < 4; ++v) fs[v] = mflux[long(p * 4 + v) * S + slot];
  } else if (kind == SSD_FACE_FARFIELD) {
    rusanov(qo, M.qinf, nx, ny, vgn, M.gamma, fs);
  } else {
    // walls: no flux relative to the (moving) wall, pressure from inside
    const float ir = 1.0f / qo[0];
    const float pr = (M.gamma - 1.0f) * (qo[3] - 0.5f * (qo[1] * qo[1] + qo[2] * qo[2]) * ir);
    fs[0] = 0.0f;
    fs[1] = pr * nx;
    fs[2] = pr * ny;
    fs[3] = pr * vgn;
  }
}

// ---------------------------------------------------------------------------
// face traces of a state held in registers
// ---------------------------------------------------------------------------
template <int N>
__device__ __forceinline__ void write_traces(const OpTables &T, const float (&Q)[4][N][N],
                                             float *__restrict__ tr, long E, int e) {
#pragma unroll
  for (int p = 0; p < N; ++p) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      float f0 = 0.f, f1 = 0.f, f2 = 0.f, f3 = 0.f;
#pragma unroll
      for (int s = 0; s < N; ++s) {
        f0 += T.I[0][s] * Q[v][s][p];   // eta = 0, point p along xi
        f2 += T.I[N][s] * Q[v][s][p];   // eta = 1
        f1 += T.I[N][s] * Q[v][p][s];   // xi = 1, point p along eta
        f3 += T.I[0][s] * Q[v][p][s];   // xi = 0
      }
      tr[long((0 * N + p) * 4 + v) * E + e] = f0;
      tr[long((1 * N + p) * 4 + v) * E + e] = f1;
      tr[long((2 * N + p) * 4 + v) * E + e] = f2;
      tr[long((3 * N + p) * 4 + v) * E + e] = f3;
    }
  }
}

template <int N>
__global__ __launch_bounds__(256) void k_traces(DevMesh M, OpTables T, const float *__restrict__ q,
                                                float *__restrict__ tr) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M.E) return;
  const long E = M.E;
  float Q[4][N][N];
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int j = 0; j < N; ++j)
#pragma unroll
      for (int i = 0; i < N; ++i) Q[v][j][i] = q[long((v * N + j) * N + i) * E + e];
  write_traces<N>(T, Q, tr, E, e);
}

// ---------------------------------------------------------------------------
// the element residual, optionally fused with an SSP-RK stage update
//   rk = false:  out = dQ/dt
//   rk = true :  out = a qn + b (q + dt dQ/dt), traces of out -> trout
// ---------------------------------------------------------------------------
template <int N, bool RK>
__global__ __launch_bounds__(256) void k_stage(DevMesh M, OpTables T, Rotation R,
                                               const float *__restrict__ q, const float *qn,
                                               float *out, const float *__restrict__ trin,
                                               float *__restrict__ trout,
                                               const float *__restrict__ mflux, float a, float b,
                                               float dt) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M.E) return;
  const long E = M.E;
  const float gm1 = M.gamma - 1.0f;

  float Q[4][N][N];
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int j = 0; j < N; ++j)
#pragma unroll
      for (int i = 0; i < N; ++i) Q[v][j][i] = q[long((v * N + j) * N + i) * E + e];

  const ElemGeo g = load_geo(M, e, R);
  uint32_t fw[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) fw[f] = M.face[long(f) * E + e];

  float res[4][N][N];
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int j = 0; j < N; ++j)
#pragma unroll
      for (int i = 0; i < N; ++i) res[v][j][i] = 0.0f;

  // ---- xi direction: rows j, flux points (Xf_k, X_j)
#pragma unroll
  for (int j = 0; j < N; ++j) {
    float Ft[4][N + 1];
#pragma unroll
    for (int k = 0; k <= N; ++k) {
      float qf[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        float acc = 0.f;
#pragma unroll
        for (int i = 0; i < N; ++i) acc += T.I[k][i] * Q[v][j][i];
        qf[v] = acc;
      }
      float nx, ny, vgn, f[4];
      metric_xi<N>(g, M, T, k, j, nx, ny, vgn);
      if (k == 0) {
        common_flux<N>(M, fw[3], j, qf, -nx, -ny, -vgn, trin, mflux, f);
#pragma unroll
        for (int v = 0; v < 4; ++v) Ft[v][k] = -f[v];
      } else if (k == N) {
        common_flux<N>(M, fw[1], j, qf, nx, ny, vgn, trin, mflux, f);
#pragma unroll
        for (int v = 0; v < 4; ++v) Ft[v][k] = f[v];
      } else {
        flux_n(qf, nx, ny, vgn, gm1, f);
#pragma unroll
        for (int v = 0; v < 4; ++v) Ft[v][k] = f[v];
      }
    }
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k <= N; ++k) acc += T.D[i][k] * Ft[v][k];
        res[v][j][i] -= acc;
      }
  }

  // ---- eta direction: columns i, flux points (X_i, Xf_k)
#pragma unroll
  for (int i = 0; i < N; ++i) {
    float Gt[4][N + 1];
#pragma unroll
    for (int k = 0; k <= N; ++k) {
      float qf[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        float acc = 0.f;
#pragma unroll
        for (int j = 0; j < N; ++j) acc += T.I[k][j] * Q[v][j][i];
        qf[v] = acc;
      }
      float nx, ny, vgn, f[4];
      metric_eta<N>(g, M, T, k, i, nx, ny, vgn);
      if (k == 0) {
        common_flux<N>(M, fw[0], i, qf, -nx, -ny, -vgn, trin, mflux, f);
#pragma unroll
        for (int v = 0; v < 4; ++v) Gt[v][k] = -f[v];
      } else if (k == N) {
        common_flux<N>(M, fw[2], i, qf, nx, ny, vgn, trin, mflux, f);
#pragma unroll
        for (int v = 0; v < 4; ++v) Gt[v][k] = f[v];
      } else {
        flux_n(qf, nx, ny, vgn, gm1, f);
#pragma unroll
        for (int v = 0; v < 4; ++v) Gt[v][k] = f[v];
      }
    }
#pragma unroll
    for (int j = 0; j < N; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k <= N; ++k) acc += T.D[j][k] * Gt[v][k];
        res[v][j][i] -= acc;
      }
  }

  // ---- dQ/dt = dQ~/dt / |J|
#pragma unroll
  for (int j = 0; j < N; ++j)
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const float ij = float(1.0 / jacobian<N>(g, M, T, j, i));
#pragma unroll
      for (int v = 0; v < 4; ++v) res[v][j][i] *= ij;
    }

  if (!RK) {
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int j = 0; j < N; ++j)
#pragma unroll
        for (int i = 0; i < N; ++i) out[long((v * N + j) * N + i) * E + e] = res[v][j][i];
    return;
  }

  // ---- SSP-RK stage: Q <- a Qn + b (Q + dt R)
  bool bad = false;
#pragma unroll
  for (int j = 0; j < N; ++j)
#pragma unroll
    for (int i = 0; i < N; ++i) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const long idx = long((v * N + j) * N + i) * E + e;
        float x = b * (Q[v][j][i] + dt * res[v][j][i]);
        if (a != 0.0f) x += a * qn[idx];
        Q[v][j][i] = x;
      }
      const float rho = Q[0][j][i];
      const float pr = gm1 * (Q[3][j][i] - 0.5f * (Q[1][j][i] * Q[1][j][i] + Q[2][j][i] * Q[2][j][i]) / rho);
      bad |= !(rho > 0.0f) || !(pr > 0.0f) || !isfinite(Q[1][j][i]) || !isfinite(Q[2][j][i]);
    }
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int j = 0; j < N; ++j)
#pragma unroll
      for (int i = 0; i < N; ++i) out[long((v * N + j) * N + i) * E + e] = Q[v][j][i];
  write_traces<N>(T, Q, trout, E, e);
  if (bad) M.flag[0] = 1;
}

// ---------------------------------------------------------------------------
// sliding interface (Sec. 3.2)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double lagrange_d(const MortarTables &MT, int N, int j, double x) {
  double r = MT.bw[j];
  for (int t = 0; t < N; ++t)
    if (t != j) r *= (x - MT.X[t]);
  return r;
}

// One workgroup: placement (m, delta) of the faces for the rotor angle and
// the 8 projection matrices.  A_k(i,j) = int_0^1 h_i(z) h_j(o_k + s_k z) dz
// by N-point Gauss-Legendre quadrature (exact: degree 2N-2).
template <int N>
__global__ __launch_bounds__(64) void k_rebuild(DevMesh M, MortarTables MT, double theta,
                                                MortarState *__restrict__ ms) {
  __shared__ double A[4][N][N];
  __shared__ double so[4], ss[4];
  if (threadIdx.x == 0) {
    const double thL = M.rotL ? theta : 0.0;
    const double thR = M.rotR ? theta : 0.0;
    const double a = (M.phi0L + thL) - (M.phi0R + thR);
    const double x = a / M.dphi;
    const double fl = floor(x);
    double d = x - fl;
    long mm = long(fl) % M.K;
    if (mm < 0) mm += M.K;
    if (d >= 1.0) {
      d = 0.0;
      mm = (mm + 1) % M.K;
    }
    so[0] = 0.0;     ss[0] = 1.0 - d;   // L face, first mortar
    so[1] = 1.0 - d; ss[1] = d;         // L face, second mortar
    so[2] = d;       ss[2] = 1.0 - d;   // R face, first mortar
    so[3] = 0.0;     ss[3] = d;         // R face, second mortar
    ms->m = int(mm);
    ms->delta = d;
    ms->thL = thL;
    ms->thR = thR;
    for (int k = 0; k < 4; ++k) {
      ms->o[k] = so[k];
      ms->s[k] = ss[k];
    }
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < 4 * N * N; idx += blockDim.x) {
    const int k = idx / (N * N), i = (idx / N) % N, j = idx % N;
    double acc = 0.0;
    for (int q = 0; q < N; ++q)
      acc += MT.wq[q] * MT.hq[q][i] * lagrange_d(MT, N, j, so[k] + ss[k] * MT.zq[q]);
    A[k][i][j] = acc;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < 4 * N * N; idx += blockDim.x) {
    const int k = idx / (N * N), i = (idx / N) % N, j = idx % N;
    double f = 0.0, bk = 0.0;
    for (int l = 0; l < N; ++l) {
      f += MT.Minv[i][l] * A[k][l][j];
      bk += MT.Minv[i][l] * A[k][j][l];
    }
    ms->Pf[k][i][j] = f;
    ms->Pb[k][i][j] = ss[k] * bk;
  }
  if (threadIdx.x == 0) ms->valid = 1;
}

template <int N>
__device__ __forceinline__ void load_canon(const DevMesh &M, const float *__restrict__ tr, int slot,
                                           double q[4][N]) {
  const long E = M.E;
  const int e = M.ring_e[slot], f = M.ring_f[slot], flip = M.ring_flip[slot];
#pragma unroll
  for (int a = 0; a < N; ++a) {
    const int pa = flip ? N - 1 - a : a;
#pragma unroll
    for (int v = 0; v < 4; ++v) q[v][a] = double(tr[long((f * N + pa) * 4 + v) * E + e]);
  }
}

// One lane per interface face (L faces 0..K-1, R faces K..2K-1).  Each lane
// forms its face's two mortars: projects both sides' traces onto the mortar
// (eq. prjQ2), takes the Rusanov flux with the exact radial normal, scales
// it to flux per unit face parameter (R_s Delta), and projects back to its
// own face (eq. prjF2).  Output: outward common flux in the element's face
// parameter order, mflux[point][var][slot].
template <int N>
__global__ __launch_bounds__(64) void k_mortar(DevMesh M, OpTables T,
                                               const MortarState *__restrict__ ms,
                                               const float *__restrict__ tr,
                                               float *__restrict__ mflux) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int K = M.K;
  if (t >= 2 * K) return;
  const bool right = t >= K;
  const int j = right ? t - K : t;
  const int m = ms->m;
  const double sc = M.Rs * M.dphi;
  double acc[4][N];
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int a = 0; a < N; ++a) acc[v][a] = 0.0;

#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int jl = right ? ((j - m - k) % K + K) % K : j;
    const int jr = right ? j : (j + m + k) % K;
    double tl[4][N], trr[4][N], ql[4][N], qr[4][N];
    load_canon<N>(M, tr, jl, tl);
    load_canon<N>(M, tr, K + jr, trr);
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int a = 0; a < N; ++a) {
        double sl = 0.0, sr = 0.0;
#pragma unroll
        for (int b = 0; b < N; ++b) {
          sl += ms->Pf[k][a][b] * tl[v][b];
          sr += ms->Pf[2 + k][a][b] * trr[v][b];
        }
        ql[v][a] = sl;
        qr[v][a] = sr;
      }
    double fm[4][N];
#pragma unroll
    for (int a = 0; a < N; ++a) {
      const double phi = M.phi0L + ms->thL + M.dphi * (jl + ms->o[k] + ms->s[k] * T.X[a]);
      double sn, cs;
      sincos(phi, &sn, &cs);
      double l4[4] = {ql[0][a], ql[1][a], ql[2][a], ql[3][a]};
      double r4[4] = {qr[0][a], qr[1][a], qr[2][a], qr[3][a]};
      double f4[4];
      rusanov_d(l4, r4, cs * sc, sn * sc, double(M.gamma), f4);
#pragma unroll
      for (int v = 0; v < 4; ++v) fm[v][a] = f4[v];
    }
    const int pb = (right ? 2 : 0) + k;
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int a = 0; a < N; ++a) {
        double s = 0.0;
#pragma unroll
        for (int b = 0; b < N; ++b) s += ms->Pb[pb][a][b] * fm[v][b];
        acc[v][a] += s;
      }
  }
  const int flip = M.ring_flip[t];
  const double sign = right ? -1.0 : 1.0;
  const long S = 2L * K;
#pragma unroll
  for (int a = 0; a < N; ++a) {
    const int pa = flip ? N - 1 - a : a;
#pragma unroll
    for (int v = 0; v < 4; ++v) mflux[long(pa * 4 + v) * S + t] = float(sign * acc[v][a]);
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
#define SSD_DISPATCH_N(N, CALL)                          \
  switch (N) {                                           \
    case 2: { constexpr int NN = 2; CALL; } break;       \
    case 3: { constexpr int NN = 3; CALL; } break;       \
    case 4: { constexpr int NN = 4; CALL; } break;       \
    case 5: { constexpr int NN = 5; CALL; } break;       \
    case 6: { constexpr int NN = 6; CALL; } break;       \
    default: return hipErrorInvalidValue;                \
  }

constexpr int STAGE_BLOCK = 128;

hipError_t launch_traces(const DevMesh &M, const OpTables &T, const float *q, float *tr,
                         hipStream_t s) {
  const int grid = (M.E + STAGE_BLOCK - 1) / STAGE_BLOCK;
  SSD_DISPATCH_N(M.N, hipLaunchKernelGGL(k_traces<NN>, dim3(grid), dim3(STAGE_BLOCK), 0, s, M, T,
                                         q, tr));
  return hipGetLastError();
}

hipError_t launch_rebuild(const DevMesh &M, const MortarTables &MT, double theta, MortarState *ms,
                          hipStream_t s) {
  SSD_DISPATCH_N(M.N, hipLaunchKernelGGL(k_rebuild<NN>, dim3(1), dim3(64), 0, s, M, MT, theta,
                                         ms));
  return hipGetLastError();
}

hipError_t launch_mortar(const DevMesh &M, const OpTables &T, const MortarState *ms,
                         const float *tr, float *mflux, hipStream_t s) {
  const int grid = (2 * M.K + 63) / 64;
  SSD_DISPATCH_N(M.N, hipLaunchKernelGGL(k_mortar<NN>, dim3(grid), dim3(64), 0, s, M, T, ms, tr,
                                         mflux));
  return hipGetLastError();
}

hipError_t launch_stage(const DevMesh &M, const OpTables &T, Rotation rot, const float *q,
                        const float *qn, float *out, const float *trin, float *trout,
                        const float *mflux, float a, float b, float dt, bool rk, hipStream_t s) {
  const int grid = (M.E + STAGE_BLOCK - 1) / STAGE_BLOCK;
  if (rk) {
    SSD_DISPATCH_N(M.N, hipLaunchKernelGGL((k_stage<NN, true>), dim3(grid), dim3(STAGE_BLOCK), 0,
                                           s, M, T, rot, q, qn, out, trin, trout, mflux, a, b,
                                           dt));
  } else {
    SSD_DISPATCH_N(M.N, hipLaunchKernelGGL((k_stage<NN, false>), dim3(grid), dim3(STAGE_BLOCK), 0,
                                           s, M, T, rot, q, qn, out, trin, trout, mflux, a, b,
                                           dt));
  }
  return hipGetLastError();
}

}  // namespace ssd

// Device-side building blocks of the SSD kernels (gfx950): buffer access,
// fluxes, element geometry and the common values at element faces.
#pragma once

#include "ssd_internal.h"

namespace ssd {

// ---------------------------------------------------------------------------
// raw buffer access: SGPR resource + per-lane byte offset + uniform byte
// offset, so address arithmetic stays on the scalar unit.  The resource
// carries the array size; the hardware returns 0 for reads past it and
// drops writes past it.
// ---------------------------------------------------------------------------
typedef __amdgpu_buffer_rsrc_t rsrc_t;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
struct f4 {
  float x[4];
};

__device__ __forceinline__ rsrc_t make_rsrc(const void *p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}
// The buffer builtins move raw 32-bit words: bit-cast, never convert.
__device__ __forceinline__ float bload(rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ void bstore(float x, rsrc_t r, uint32_t voff, uint32_t soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, x), r, voff, soff, 0);
}
__device__ __forceinline__ f4 bload4(rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}
__device__ __forceinline__ void bstore4(const float x[4], rsrc_t r, uint32_t voff, uint32_t soff) {
  f4 t;
#pragma unroll
  for (int v = 0; v < 4; ++v) t.x[v] = x[v];
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, t), r, voff, soff, 0);
}

// Streaming forms: the non-temporal cache policy (bit 1 of the policy
// operand on gfx950), for large arrays a kernel touches once, so that they
// do not push out of the caches what this or the next kernel reads again.
constexpr int kNT = 2;
__device__ __forceinline__ float bload_nt(rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, kNT));
}
__device__ __forceinline__ void bstore_nt(float x, rsrc_t r, uint32_t voff, uint32_t soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, x), r, voff, soff, kNT);
}

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// A wave-uniform float as an opaque register value.
__device__ __forceinline__ float uniform(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, x)));
}

// Number of set bits of the wave mask m below the calling lane.
__device__ __forceinline__ int lane_rank(uint64_t m) {
  return int(__builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u)));
}

// ---------------------------------------------------------------------------
// fluxes (Sec. 2.1, 2.2, 3.1)
// ---------------------------------------------------------------------------
// Normal inviscid ALE flux along the scaled normal (nx, ny):
// (F - u_g Q) nx + (G - v_g Q) ny with vgn = u_g nx + v_g ny.
__device__ __forceinline__ void flux_n(const float q[4], float nx, float ny, float vgn, float gm1,
                                       float f[4]) {
  const float ir = rcp(q[0]);
  const float u = q[1] * ir, v = q[2] * ir;
  const float p = gm1 * (q[3] - 0.5f * (q[1] * u + q[2] * v));
  const float un = u * nx + v * ny;
  const float rel = un - vgn;
  f[0] = q[0] * rel;
  f[1] = q[1] * rel + p * nx;
  f[2] = q[2] * rel + p * ny;
  f[3] = q[3] * rel + p * un;
}

// Rusanov common flux from the owner (l) towards the neighbour (r); *p_own
// receives the owner's pressure.
__device__ __forceinline__ void rusanov(const float ql[4], const float qr[4], float nx, float ny,
                                        float vgn, float gam, float f[4], float *p_own = nullptr) {
  const float gm1 = gam - 1.0f;
  const float n2 = nx * nx + ny * ny;
  const float irl = rcp(ql[0]), irr = rcp(qr[0]);
  const float ul = ql[1] * irl, vl = ql[2] * irl;
  const float ur = qr[1] * irr, vr = qr[2] * irr;
  const float pl = gm1 * (ql[3] - 0.5f * (ql[1] * ul + ql[2] * vl));
  const float pr = gm1 * (qr[3] - 0.5f * (qr[1] * ur + qr[2] * vr));
  if (p_own) *p_own = pl;
  const float unl = ul * nx + vl * ny, unr = ur * nx + vr * ny;
  const float rl = unl - vgn, rr = unr - vgn;
  // c |n| of each side as one root: sqrt(gamma p / rho |n|^2)
  const float cnl = __builtin_amdgcn_sqrtf(gam * pl * irl * n2);
  const float cnr = __builtin_amdgcn_sqrtf(gam * pr * irr * n2);
  const float lam = fmaxf(fabsf(rl) + cnl, fabsf(rr) + cnr);
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

// Gas constants of the viscous terms: mu, and kT = k (gamma - 1) / R =
// mu gamma / Pr, the conductivity k = mu gamma R / ((gamma - 1) Pr) times
// the factor that turns the gradient of the specific internal energy into
// the gradient of T.
struct ViscParams {
  float mu, kT;
};

__device__ __forceinline__ ViscParams visc_params(const DevMesh &M) {
  ViscParams P;
  P.mu = M.mu;
  P.kT = M.mu * M.gamma * rcp(M.prandtl);
  return P;
}

// 1 / x: the hardware reciprocal in FP32 (within 1 ulp), a division in FP64.
__device__ __forceinline__ float recip(float x) { return rcp(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

// Normal viscous flux F_vis nx + G_vis ny (Sec. 2.1) from the conservative
// state and its x, y gradients: tau_ij = mu (u_i,j + u_j,i) - 2/3 mu
// delta_ij div u and the heat flux k grad T, T = p / (rho R).  In the
// conservative gradients, with E = rho E / rho and g_c = grad Q_c . n,
//   rho grad u = grad(rho u) - u grad rho   (likewise v),
//   k grad T . n = (kT / rho) (g_3 - u g_1 - v g_2 + (|u|^2 - E) g_0),
// kT = k (gamma - 1) / R; the energy row is -(u (tau n)_x + v (tau n)_y +
// k grad T . n).
template <typename R>
__device__ __forceinline__ void visc_flux_n(const R q[4], const R gx[4], const R gy[4], R nx, R ny,
                                            R mu, R kT, R f[4]) {
  const R ir = recip(q[0]);
  const R u = q[1] * ir, v = q[2] * ir;
  const R mir = mu * ir;
  // mu times the velocity gradients
  const R ux = (gx[1] - u * gx[0]) * mir, vx = (gx[2] - v * gx[0]) * mir;
  const R uy = (gy[1] - u * gy[0]) * mir, vy = (gy[2] - v * gy[0]) * mir;
  const R txy = uy + vx;
  const R txx = R(2.0 / 3.0) * (R(2) * ux - vy);
  const R tyy = R(2.0 / 3.0) * (R(2) * vy - ux);
  const R s1 = txx * nx + txy * ny, s2 = txy * nx + tyy * ny;
  R g[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) g[c] = gx[c] * nx + gy[c] * ny;
  const R w = u * u + v * v - q[3] * ir;
  const R h = g[3] - u * g[1] - v * g[2] + w * g[0];
  f[0] = R(0);
  f[1] = -s1;
  f[2] = -s2;
  f[3] = -(u * s1 + v * s2 + kT * ir * h);
}

// ---------------------------------------------------------------------------
// element geometry (Sec. 2.3).  A bilinear cell is x(xi, eta) = p0 + xi A +
// eta C + xi eta T with corner 0 at p0, edges A = x3 - x0, C = x9 - x0 and
// twist T = x6 - x3 - x9 + x0; the host differences them in FP64 and stores
// them in FP32 (8 floats per cell, all cells).  They are rotated once into
// the current frame, so every metric is a linear combination:
//   x_xi(eta) = A + eta T,  x_eta(xi) = C + xi T.
// Cubic cells read FP64 tables and rotate in FP64.
// ---------------------------------------------------------------------------
struct ElemGeo {
  int cubic, c;
  float w;                                    // omega of the zone (0: fixed)
  float p0x, p0y, Ax, Ay, Cx, Cy, Tx, Ty;
  double ct, st;
};

__device__ __forceinline__ ElemGeo load_geo(const DevMesh &M, int e, const Rotation &R) {
  ElemGeo g;
  const long E = M.E;
  // the edge vectors are read for every cell (cubic cells ignore them) so
  // that no load waits on the flag word
  float v[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) v[k] = M.geo[cb_index32(uint32_t(e), k, 8u, uint32_t(E))];
  const int fl = M.eflag[e];
  g.cubic = fl & EF_CUBIC;
  g.c = fl >> 8;
  const bool rot = (fl & EF_ROT) != 0;
  g.ct = rot ? R.ct : 1.0;
  g.st = rot ? R.st : 0.0;
  g.w = rot ? float(R.omega) : 0.0f;
  const float c = float(g.ct), s = float(g.st);
  g.p0x = c * v[0] - s * v[1];   g.p0y = s * v[0] + c * v[1];
  g.Ax = c * v[2] - s * v[3];    g.Ay = s * v[2] + c * v[3];
  g.Cx = c * v[4] - s * v[5];    g.Cy = s * v[4] + c * v[5];
  g.Tx = c * v[6] - s * v[7];    g.Ty = s * v[6] + c * v[7];
  return g;
}

// Metric data of one flux point: scaled normal (nx, ny) of the flux-point
// line, u_g . n, and the grid velocity (ug, vg) there (zero on fixed cells).
struct FPGeo {
  float nx, ny, vgn, ug, vg;
};

// Metric data of a bilinear cell along one line of flux points, as
// polynomials in the line parameter t: the scaled normal is linear in t, the
// position (for the grid velocity) linear, and u_g . n quadratic.  Built
// once per line, then two fused multiply-adds per quantity and point.
struct LineGeo {
  float n0x, n1x, n0y, n1y;   // n(t) = n0 + t n1
  float p0x, p1x, p0y, p1y;   // position x(t) = p0 + t p1 (current frame)
  float v0, v1, v2;           // u_g . n = v0 + t (v1 + t v2)
  float w;                    // omega of the zone (0: fixed)
};

// xi-direction line at eta: n = (y_eta, -x_eta), x_eta(xi) = C + xi (D - C),
// u_g . n = -w (x . x_eta + y . y_eta).
__device__ __forceinline__ LineGeo line_xi(const ElemGeo &g, float eta) {
  LineGeo L;
  const float ex0 = g.Cx, ex1 = g.Tx, ey0 = g.Cy, ey1 = g.Ty;
  L.n0x = ey0;
  L.n1x = ey1;
  L.n0y = -ex0;
  L.n1y = -ex1;
  L.p0x = g.p0x + eta * g.Cx;
  L.p1x = g.Ax + eta * g.Tx;
  L.p0y = g.p0y + eta * g.Cy;
  L.p1y = g.Ay + eta * g.Ty;
  L.w = g.w;
  L.v0 = -g.w * (L.p0x * ex0 + L.p0y * ey0);
  L.v1 = -g.w * (L.p0x * ex1 + L.p1x * ex0 + L.p0y * ey1 + L.p1y * ey0);
  L.v2 = -g.w * (L.p1x * ex1 + L.p1y * ey1);
  return L;
}

// eta-direction line at xi: n = (-y_xi, x_xi), x_xi(eta) = A + eta (B - A),
// u_g . n = w (x . x_xi + y . y_xi).
__device__ __forceinline__ LineGeo line_eta(const ElemGeo &g, float xi) {
  LineGeo L;
  const float ex0 = g.Ax, ex1 = g.Tx, ey0 = g.Ay, ey1 = g.Ty;
  L.n0x = -ey0;
  L.n1x = -ey1;
  L.n0y = ex0;
  L.n1y = ex1;
  L.p0x = g.p0x + xi * g.Ax;
  L.p1x = g.Cx + xi * g.Tx;
  L.p0y = g.p0y + xi * g.Ay;
  L.p1y = g.Cy + xi * g.Ty;
  L.w = g.w;
  L.v0 = g.w * (L.p0x * ex0 + L.p0y * ey0);
  L.v1 = g.w * (L.p0x * ex1 + L.p1x * ex0 + L.p0y * ey1 + L.p1y * ey0);
  L.v2 = g.w * (L.p1x * ex1 + L.p1y * ey1);
  return L;
}

__device__ __forceinline__ FPGeo line_at(const LineGeo &L, float t) {
  FPGeo r;
  r.nx = L.n0x + t * L.n1x;
  r.ny = L.n0y + t * L.n1y;
  r.vgn = L.v0 + t * (L.v1 + t * L.v2);
  r.ug = -L.w * (L.p0y + t * L.p1y);
  r.vg = L.w * (L.p0x + t * L.p1x);
  return r;
}

// xi-direction flux point (Xf_k, X_j): n = (y_eta, -x_eta) in the current
// frame; L = line_xi(g, X_j) for bilinear cells.
template <int N>
__device__ __forceinline__ FPGeo metric_xi(const ElemGeo &g, const LineGeo &L, const DevMesh &M,
                                           const OpTables &T, int k, int j) {
  if (g.cubic) {
    FPGeo r;
    r.ug = r.vg = r.vgn = 0.0f;
    const double xe = M.cmet[cubic_xi_index(N, M.C, 0, j, k, g.c)];
    const double ye = M.cmet[cubic_xi_index(N, M.C, 1, j, k, g.c)];
    r.nx = float(g.st * xe + g.ct * ye);
    r.ny = float(-(g.ct * xe - g.st * ye));
    if (g.w != 0.0f) {
      const double px = M.cmet[cubic_xi_index(N, M.C, 2, j, k, g.c)];
      const double py = M.cmet[cubic_xi_index(N, M.C, 3, j, k, g.c)];
      r.vgn = float(-double(g.w) * (px * xe + py * ye));
      r.ug = float(-double(g.w) * (g.st * px + g.ct * py));
      r.vg = float(double(g.w) * (g.ct * px - g.st * py));
    }
    return r;
  }
  return line_at(L, float(T.Xf[k]));
}

// eta-direction flux point (X_i, Xf_k): n = (-y_xi, x_xi) in the current
// frame; L = line_eta(g, X_i) for bilinear cells.
template <int N>
__device__ __forceinline__ FPGeo metric_eta(const ElemGeo &g, const LineGeo &L, const DevMesh &M,
                                            const OpTables &T, int k, int i) {
  if (g.cubic) {
    FPGeo r;
    r.ug = r.vg = r.vgn = 0.0f;
    const double xx = M.cmet[cubic_eta_index(N, M.C, 0, k, i, g.c)];
    const double yx = M.cmet[cubic_eta_index(N, M.C, 1, k, i, g.c)];
    r.nx = float(-(g.st * xx + g.ct * yx));
    r.ny = float(g.ct * xx - g.st * yx);
    if (g.w != 0.0f) {
      const double px = M.cmet[cubic_eta_index(N, M.C, 2, k, i, g.c)];
      const double py = M.cmet[cubic_eta_index(N, M.C, 3, k, i, g.c)];
      r.vgn = float(double(g.w) * (px * xx + py * yx));
      r.ug = float(-double(g.w) * (g.st * px + g.ct * py));
      r.vg = float(double(g.w) * (g.ct * px - g.st * py));
    }
    return r;
  }
  return line_at(L, float(T.Xf[k]));
}

// Metric derivatives x_xi, y_xi, x_eta, y_eta at the solution point
// (X_i, X_j) in the current frame, and 1 / |J|.
struct SPGeo {
  float xx, yx, xe, ye, ij;
};

template <int N>
__device__ __forceinline__ SPGeo metric_sp(const ElemGeo &g, const DevMesh &M, const OpTables &T,
                                           int j, int i) {
  SPGeo r;
  if (g.cubic) {
    const double J = M.cmet[cubic_sp_index(N, M.C, 0, j, i, g.c)];
    const double xx = M.cmet[cubic_sp_index(N, M.C, 1, j, i, g.c)];
    const double xe = M.cmet[cubic_sp_index(N, M.C, 2, j, i, g.c)];
    const double yx = M.cmet[cubic_sp_index(N, M.C, 3, j, i, g.c)];
    const double ye = M.cmet[cubic_sp_index(N, M.C, 4, j, i, g.c)];
    r.xx = float(g.ct * xx - g.st * yx);
    r.yx = float(g.st * xx + g.ct * yx);
    r.xe = float(g.ct * xe - g.st * ye);
    r.ye = float(g.st * xe + g.ct * ye);
    r.ij = float(1.0 / J);
    return r;
  }
  const float xi = float(T.X[i]), eta = float(T.X[j]);
  r.xx = g.Ax + eta * g.Tx;
  r.yx = g.Ay + eta * g.Ty;
  r.xe = g.Cx + xi * g.Tx;
  r.ye = g.Cy + xi * g.Ty;
  r.ij = rcp(r.xx * r.ye - r.xe * r.yx);
  return r;
}

// 1 / |J| at the solution point (X_i, X_j).
template <int N>
__device__ __forceinline__ float inv_jacobian(const ElemGeo &g, const DevMesh &M,
                                              const OpTables &T, int j, int i) {
  if (g.cubic) return float(1.0 / M.cmet[cubic_sp_index(N, M.C, 0, j, i, g.c)]);
  const float xi = float(T.X[i]), eta = float(T.X[j]);
  const float xx = g.Ax + eta * g.Tx, yx = g.Ay + eta * g.Ty;
  const float xe = g.Cx + xi * g.Tx, ye = g.Cy + xi * g.Ty;
  return rcp(xx * ye - xe * yx);
}

// ---------------------------------------------------------------------------
// face data
// ---------------------------------------------------------------------------
// What a face needs from outside the block, fetched before it is used: the
// neighbour's trace (a face without the in-block bit), the far-field state, or
// the interface record (projected mortar flux, or projected common
// solution) of a sliding face.  Traces and interface records share one face
// data buffer (rface, `bytes` long), the records from byte `side_base`.
// In-block faces, and walls, need nothing: their
// lanes point the load past the end of the buffer, where a buffer load
// returns zero without a memory access.  One load per lane, no branch.
template <int N>
__device__ __forceinline__ void prefetch_face(const DevMesh &M, rsrc_t rface, uint32_t bytes,
                                              uint32_t side_base, uint32_t E, uint32_t fw, int p,
                                              float x[4]) {
  const int kind = face_kind_of(fw);
  const uint32_t idx = uint32_t(face_idx_of(fw)), nf = uint32_t(face_nf_of(fw));
  const uint32_t pp = face_rev_of(fw) ? uint32_t(N - 1 - p) : uint32_t(p);
  const bool from_trace =
      (kind == SSD_FACE_INTERIOR || kind == SSD_FACE_PERIODIC) && !face_inblock_of(fw);
  const uint32_t off = from_trace ? ((nf * E + idx) * N + pp) * 16u
                       : kind == SSD_FACE_SLIDING ? side_base + (idx * N + uint32_t(p)) * 16u
                                                  : bytes;
  const f4 a = bload4(rface, off, 0u);
#pragma unroll
  for (int v = 0; v < 4; ++v) x[v] = a.x[v];
  if (__builtin_expect(kind == SSD_FACE_FARFIELD, 0)) {
#pragma unroll
    for (int v = 0; v < 4; ++v) x[v] = M.qinf[v];
  }
}

__device__ __forceinline__ bool conforming(int kind) {
  return kind == SSD_FACE_INTERIOR || kind == SSD_FACE_PERIODIC;
}

// The neighbour's solution at the face point matching point p of face word
// fw: interpolated from the block's LDS state Sf [var][j][i][lane] for an
// in-block face, else the prefetched value.
template <int N>
__device__ __forceinline__ void neighbor_state(const OpTables &T, const float *Sf, uint32_t fw,
                                               int p, const float x[4], float qx[4]) {
  if (face_inblock_of(fw)) {
    const uint32_t nf = uint32_t(face_nf_of(fw));
    const int pp = face_rev_of(fw) ? N - 1 - p : p;
    const int ln = face_idx_of(fw) & (EB - 1);
    const bool odd = (nf & 1u) != 0;               // xi faces: the point runs along eta
    const bool hi = (nf == 1u || nf == 2u);        // xi = 1 or eta = 1
    const int base = (odd ? pp * N * EB : pp * EB) + ln;
    const int stride = odd ? EB : N * EB;
    // the weights are uniform values selected per lane; taken through
    // readfirstlane so that the selection stays a register select instead
    // of becoming a per-lane load from the kernel argument segment
    float wgt[N];
#pragma unroll
    for (int s2 = 0; s2 < N; ++s2) {
      const float a0 = uniform(T.I[0][s2]), aN = uniform(T.I[N][s2]);
      wgt[s2] = hi ? aN : a0;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      float acc = 0.f;
#pragma unroll
      for (int s2 = 0; s2 < N; ++s2) acc += wgt[s2] * Sf[v * N * N * EB + base + s2 * stride];
      qx[v] = acc;
    }
  } else {
#pragma unroll
    for (int v = 0; v < 4; ++v) qx[v] = x[v];
  }
}

// Orders whose inviscid stage passes the solution traces at a line's two
// end points between the block's elements through LDS: the exchange array,
// [side][4][N][64] floats (8 KB at N = 4), keeps the block at 4 per compute
// unit, as without it.
template <int N>
__device__ constexpr bool trace_shared() {
  return N <= 4;
}

// neighbor_state with the exchange array X (XCH): an in-block neighbour's
// trace at point p comes from the same wave (row phase: row p; column
// phase: column p), which has written it to X before; four LDS reads instead
// of an interpolation of the neighbour's line.
template <int N, bool XCH>
__device__ __forceinline__ void neighbor_state_x(const OpTables &T, const float *Sf, const float *X,
                                                 uint32_t fw, int p, const float x[4],
                                                 float qx[4]) {
  if (!XCH) {
    neighbor_state<N>(T, Sf, fw, p, x, qx);
  } else if (face_inblock_of(fw)) {
    const uint32_t nf = uint32_t(face_nf_of(fw));
    const int side = (nf == 1u || nf == 2u) ? 1 : 0;   // xi = 1 / eta = 1
    const float *xs = X + (side * 4 * N + p) * EB + (face_idx_of(fw) & (EB - 1));
#pragma unroll
    for (int v = 0; v < 4; ++v) qx[v] = xs[v * N * EB];
  } else {
#pragma unroll
    for (int v = 0; v < 4; ++v) qx[v] = x[v];
  }
}

// Common inviscid normal flux at one element-boundary flux point along the
// outward normal of `G`, given the state across the face qx (the
// neighbour's on conforming faces, the far-field state on far-field faces)
// and the face data x (see prefetch_face).  The Rusanov flux is formed for
// every lane; walls and sliding faces replace it in a branch that the waves
// without such faces (most of them) skip.
__device__ __forceinline__ void common_flux(const DevMesh &M, uint32_t fw, const float qo[4],
                                            const float qx[4], const float x[4], const FPGeo &G,
                                            float fs[4]) {
  const int kind = face_kind_of(fw);
  float fr[4], pr;
  rusanov(qo, qx, G.nx, G.ny, G.vgn, M.gamma, fr, &pr);
  // walls: no flux relative to the moving wall; pressure from the interior
  const bool wall = kind == SSD_FACE_WALL_ISOTHERMAL || kind == SSD_FACE_WALL_SLIP;
  const bool sliding = kind == SSD_FACE_SLIDING;
#pragma unroll
  for (int v = 0; v < 4; ++v) fs[v] = fr[v];
  if (__builtin_expect(wall || sliding, 0)) {
    const float fw4[4] = {0.0f, pr * G.nx, pr * G.ny, pr * G.vgn};
#pragma unroll
    for (int v = 0; v < 4; ++v) fs[v] = sliding ? x[v] : fw4[v];
  }
}

// Common solution at a face point for the gradient (BR1 reading): the mean
// of both sides on conforming faces; the wall state on isothermal walls
// (interior pressure, wall temperature, wall velocity = grid velocity);
// the interior state without its normal velocity relative to the wall on
// slip walls; the far-field state; the projected mortar value on sliding
// faces (x).  qx is the neighbour's state on conforming faces.
__device__ __forceinline__ void common_solution(const DevMesh &M, int kind, const float qo[4],
                                                const float qx[4], const float x[4],
                                                const FPGeo &G, float qc[4]) {
  if (kind == SSD_FACE_INTERIOR || kind == SSD_FACE_PERIODIC) {
#pragma unroll
    for (int v = 0; v < 4; ++v) qc[v] = 0.5f * (qo[v] + qx[v]);
    return;
  }
  if (kind == SSD_FACE_SLIDING || kind == SSD_FACE_FARFIELD) {
#pragma unroll
    for (int v = 0; v < 4; ++v) qc[v] = x[v];
    return;
  }
  const float gm1 = M.gamma - 1.0f;
  const float ir = rcp(qo[0]);
  const float u = qo[1] * ir, v = qo[2] * ir;
  const float p = gm1 * (qo[3] - 0.5f * (qo[1] * u + qo[2] * v));
  const float igm1 = rcp(gm1);
  if (kind == SSD_FACE_WALL_ISOTHERMAL) {
    const float rb = p * rcp(M.gas_R * M.T_wall);
    qc[0] = rb;
    qc[1] = rb * G.ug;
    qc[2] = rb * G.vg;
    qc[3] = p * igm1 + 0.5f * rb * (G.ug * G.ug + G.vg * G.vg);
    return;
  }
  // slip wall
  const float im = rcp(__builtin_amdgcn_sqrtf(G.nx * G.nx + G.ny * G.ny));
  const float hx = G.nx * im, hy = G.ny * im;
  const float un = (u - G.ug) * hx + (v - G.vg) * hy;
  const float ub = u - un * hx, vb = v - un * hy;
  qc[0] = qo[0];
  qc[1] = qo[0] * ub;
  qc[2] = qo[0] * vb;
  qc[3] = p * igm1 + 0.5f * qo[0] * (ub * ub + vb * vb);
}

}  // namespace ssd

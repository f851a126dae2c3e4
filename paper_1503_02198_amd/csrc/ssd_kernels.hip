// HIP kernels of the SSD residual for gfx950 (CDNA4).
//
// Layout: SoA with the element index fastest, so a wave that serves 64
// consecutive elements reads and writes contiguous 256-byte rows per
// (variable, point).  Face traces (the solution interpolated to the
// element-boundary flux points) travel between blocks through a trace buffer
// laid out [face][element][point][var]: one lane moves the 4 variables of a
// point as one 16-byte access, and the N waves of a block together touch
// whole 16 N-byte face records.
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
  const float ir = __builtin_amdgcn_rcpf(q[0]);
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
  const float mag = __builtin_amdgcn_sqrtf(nx * nx + ny * ny);
  const float irl = __builtin_amdgcn_rcpf(ql[0]), irr = __builtin_amdgcn_rcpf(qr[0]);
  const float ul = ql[1] * irl, vl = ql[2] * irl;
  const float ur = qr[1] * irr, vr = qr[2] * irr;
  const float pl = gm1 * (ql[3] - 0.5f * (ql[1] * ul + ql[2] * vl));
  const float pr = gm1 * (qr[3] - 0.5f * (qr[1] * ur + qr[2] * vr));
  const float unl = ul * nx + vl * ny, unr = ur * nx + vr * ny;
  const float rl = unl - vgn, rr = unr - vgn;
  const float cl = __builtin_amdgcn_sqrtf(gam * pl * irl), cr = __builtin_amdgcn_sqrtf(gam * pr * irr);
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
// raw buffer access: SGPR resource + per-lane byte offset + uniform byte
// offset, so address arithmetic stays on the scalar unit.  The resource
// carries the array size; the hardware returns 0 for reads past it and
// drops writes past it.
// ---------------------------------------------------------------------------
typedef __amdgpu_buffer_rsrc_t rsrc_t;

__device__ __forceinline__ rsrc_t make_rsrc(const void *p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
struct f4 {
  float x[4];
};

// The buffer builtins move raw 32-bit words: bit-cast, never convert.
__device__ __forceinline__ f4 bload4(rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}
__device__ __forceinline__ void bstore4(const float x[4], rsrc_t r, uint32_t voff, uint32_t soff) {
  f4 t;
#pragma unroll
  for (int v = 0; v < 4; ++v) t.x[v] = x[v];
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, t), r, voff, soff, 0);
}
__device__ __forceinline__ float bload(rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ void bstore(float x, rsrc_t r, uint32_t voff, uint32_t soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, x), r, voff, soff, 0);
}

// ---------------------------------------------------------------------------
// element geometry (Sec. 2.3).  Bilinear cells: the four edge vectors are
// differenced in FP64 from the stored corners, then carried in FP32 and
// rotated once into the current frame, so every metric is a linear
// combination:  x_xi(eta) = A + eta (B - A),  x_eta(xi) = C + xi (D - C),
// x(xi, eta) = p0 + xi A + eta C + xi eta (B - A).  Cubic cells read FP64
// tables and rotate in FP64.
// ---------------------------------------------------------------------------
struct ElemGeo {
  int cubic, c;
  float w;                                    // omega of the zone (0: fixed)
  float p0x, p0y, Ax, Ay, Bx, By, Cx, Cy, Dx, Dy;
  double ct, st;
};

__device__ __forceinline__ ElemGeo load_geo(const DevMesh &M, int e, const Rotation &R) {
  ElemGeo g;
  const long E = M.E;
  // corners are read for every cell (cubic cells ignore them) so that no
  // load waits on the flag word
  const double x0 = M.corners[0 * E + e], y0 = M.corners[1 * E + e];
  const double x3 = M.corners[2 * E + e], y3 = M.corners[3 * E + e];
  const double x6 = M.corners[4 * E + e], y6 = M.corners[5 * E + e];
  const double x9 = M.corners[6 * E + e], y9 = M.corners[7 * E + e];
  const int fl = M.eflag[e];
  g.cubic = fl & EF_CUBIC;
  g.c = fl >> 8;
  const bool rot = (fl & EF_ROT) != 0;
  g.ct = rot ? R.ct : 1.0;
  g.st = rot ? R.st : 0.0;
  g.w = rot ? float(R.omega) : 0.0f;
  const float c = float(g.ct), s = float(g.st);
  auto rx = [&](double x, double y) { return c * float(x) - s * float(y); };
  auto ry = [&](double x, double y) { return s * float(x) + c * float(y); };
  g.p0x = rx(x0, y0);            g.p0y = ry(x0, y0);
  g.Ax = rx(x3 - x0, y3 - y0);   g.Ay = ry(x3 - x0, y3 - y0);
  g.Bx = rx(x6 - x9, y6 - y9);   g.By = ry(x6 - x9, y6 - y9);
  g.Cx = rx(x9 - x0, y9 - y0);   g.Cy = ry(x9 - x0, y9 - y0);
  g.Dx = rx(x6 - x3, y6 - y3);   g.Dy = ry(x6 - x3, y6 - y3);
  return g;
}

// Scaled normal (y_eta, -x_eta) at the xi-direction flux point (Xf_k, X_j)
// in the current frame, and u_g . n.
template <int N>
__device__ __forceinline__ void metric_xi(const ElemGeo &g, const DevMesh &M, const OpTables &T,
                                          int k, int j, float &nx, float &ny, float &vgn) {
  if (g.cubic) {
    const double xe = M.cmet[cubic_xi_index(N, M.C, 0, j, k, g.c)];
    const double ye = M.cmet[cubic_xi_index(N, M.C, 1, j, k, g.c)];
    double v = 0.0;
    if (g.w != 0.0f)
      v = -double(g.w) * (M.cmet[cubic_xi_index(N, M.C, 2, j, k, g.c)] * xe +
                          M.cmet[cubic_xi_index(N, M.C, 3, j, k, g.c)] * ye);
    nx = float(g.st * xe + g.ct * ye);
    ny = float(-(g.ct * xe - g.st * ye));
    vgn = float(v);
    return;
  }
  const float xi = float(T.Xf[k]), eta = float(T.X[j]);
  const float xe = g.Cx + xi * (g.Dx - g.Cx), ye = g.Cy + xi * (g.Dy - g.Cy);
  nx = ye;
  ny = -xe;
  vgn = 0.0f;
  if (g.w != 0.0f) {
    const float px = g.p0x + xi * g.Ax + eta * g.Cx + xi * eta * (g.Bx - g.Ax);
    const float py = g.p0y + xi * g.Ay + eta * g.Cy + xi * eta * (g.By - g.Ay);
    vgn = -g.w * (px * xe + py * ye);
  }
}

// Scaled normal (-y_xi, x_xi) at the eta-direction flux point (X_i, Xf_k).
template <int N>
__device__ __forceinline__ void metric_eta(const ElemGeo &g, const DevMesh &M, const OpTables &T,
                                           int k, int i, float &nx, float &ny, float &vgn) {
  if (g.cubic) {
    const double xx = M.cmet[cubic_eta_index(N, M.C, 0, k, i, g.c)];
    const double yx = M.cmet[cubic_eta_index(N, M.C, 1, k, i, g.c)];
    double v = 0.0;
    if (g.w != 0.0f)
      v = double(g.w) * (M.cmet[cubic_eta_index(N, M.C, 2, k, i, g.c)] * xx +
                         M.cmet[cubic_eta_index(N, M.C, 3, k, i, g.c)] * yx);
    nx = float(-(g.st * xx + g.ct * yx));
    ny = float(g.ct * xx - g.st * yx);
    vgn = float(v);
    return;
  }
  const float xi = float(T.X[i]), eta = float(T.Xf[k]);
  const float xx = g.Ax + eta * (g.Bx - g.Ax), yx = g.Ay + eta * (g.By - g.Ay);
  nx = -yx;
  ny = xx;
  vgn = 0.0f;
  if (g.w != 0.0f) {
    const float px = g.p0x + xi * g.Ax + eta * g.Cx + xi * eta * (g.Bx - g.Ax);
    const float py = g.p0y + xi * g.Ay + eta * g.Cy + xi * eta * (g.By - g.Ay);
    vgn = g.w * (px * xx + py * yx);
  }
}

// 1 / |J| at the solution point (X_i, X_j).
template <int N>
__device__ __forceinline__ float inv_jacobian(const ElemGeo &g, const DevMesh &M,
                                              const OpTables &T, int j, int i) {
  if (g.cubic) return float(1.0 / M.cmet[cubic_sp_index(N, M.C, 0, j, i, g.c)]);
  const float xi = float(T.X[i]), eta = float(T.X[j]);
  const float xx = g.Ax + eta * (g.Bx - g.Ax), yx = g.Ay + eta * (g.By - g.Ay);
  const float xe = g.Cx + xi * (g.Dx - g.Cx), ye = g.Cy + xi * (g.Dy - g.Cy);
  return __builtin_amdgcn_rcpf(xx * ye - xe * yx);
}

// ---------------------------------------------------------------------------
// common normal flux at one element-boundary flux point (outward normal)
// ---------------------------------------------------------------------------
struct StageBufs {
  rsrc_t q, qn, out, trin, trout, mflux;
  uint32_t E4;      // bytes per state row (4 E)
  uint32_t S4;      // bytes per mortar-flux row (4 * 2K)
};

// What a face needs from outside the block, fetched before it is used:
// the neighbour's trace (a neighbour in another block), the far-field state,
// or the projected mortar flux (a sliding face).  Faces whose neighbour is in
// the same block, and walls, fetch nothing.
template <int N>
__device__ __forceinline__ void prefetch_face(const DevMesh &M, const StageBufs &B, uint32_t fw,
                                              int p, float x[4]) {
  const int kind = face_kind_of(fw);
#pragma unroll
  for (int v = 0; v < 4; ++v) x[v] = 0.0f;
  if (kind == SSD_FACE_SLIDING) {
    const f4 t = bload4(B.mflux, (uint32_t(face_idx_of(fw)) * N + uint32_t(p)) * 16u, 0u);
#pragma unroll
    for (int v = 0; v < 4; ++v) x[v] = t.x[v];
  } else if (kind == SSD_FACE_FARFIELD) {
#pragma unroll
    for (int v = 0; v < 4; ++v) x[v] = M.qinf[v];
  } else if ((kind == SSD_FACE_INTERIOR || kind == SSD_FACE_PERIODIC) && !face_inblock_of(fw)) {
    const uint32_t nb = uint32_t(face_idx_of(fw)), nf = uint32_t(face_nf_of(fw));
    const uint32_t pp = face_rev_of(fw) ? uint32_t(N - 1 - p) : uint32_t(p);
    const f4 t = bload4(B.trin, ((nf * (B.E4 >> 2) + nb) * N + pp) * 16u, 0u);
#pragma unroll
    for (int v = 0; v < 4; ++v) x[v] = t.x[v];
  }
}

// Common normal flux at one element-boundary flux point along the outward
// normal (nx, ny), given the prefetched face data x.  A neighbour in the
// same block is interpolated from the block's LDS state Sf [var][j][i][lane].
template <int N>
__device__ __forceinline__ void common_flux(const DevMesh &M, const OpTables &T, const float *Sf,
                                            uint32_t fw, int p, const float qo[4],
                                            const float x[4], float nx, float ny, float vgn,
                                            float fs[4]) {
  const int kind = face_kind_of(fw);
  if (kind == SSD_FACE_SLIDING) {
#pragma unroll
    for (int v = 0; v < 4; ++v) fs[v] = x[v];
    return;
  }
  if (kind == SSD_FACE_WALL_ISOTHERMAL || kind == SSD_FACE_WALL_SLIP) {
    // no flux relative to the moving wall; pressure from the interior
    const float pr = (M.gamma - 1.0f) *
                     (qo[3] - 0.5f * (qo[1] * qo[1] + qo[2] * qo[2]) * __builtin_amdgcn_rcpf(qo[0]));
    fs[0] = 0.0f;
    fs[1] = pr * nx;
    fs[2] = pr * ny;
    fs[3] = pr * vgn;
    return;
  }
  float qx[4];
  if ((kind == SSD_FACE_INTERIOR || kind == SSD_FACE_PERIODIC) && face_inblock_of(fw)) {
    const uint32_t nf = uint32_t(face_nf_of(fw));
    const int pp = face_rev_of(fw) ? N - 1 - p : p;
    const int ln = face_idx_of(fw) & (EB - 1);
    const bool odd = (nf & 1u) != 0;               // xi faces: the point runs along eta
    const bool hi = (nf == 1u || nf == 2u);        // xi = 1 or eta = 1
    const int base = (odd ? pp * N * EB : pp * EB) + ln;
    const int stride = odd ? EB : N * EB;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      float acc = 0.f;
#pragma unroll
      for (int s2 = 0; s2 < N; ++s2)
        acc += (hi ? T.I[N][s2] : T.I[0][s2]) * Sf[v * N * N * EB + base + s2 * stride];
      qx[v] = acc;
    }
  } else {
#pragma unroll
    for (int v = 0; v < 4; ++v) qx[v] = x[v];
  }
  rusanov(qo, qx, nx, ny, vgn, M.gamma, fs);
}

// ---------------------------------------------------------------------------
// face traces of a state, for the faces some other block reads
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(256) void k_traces(DevMesh M, OpTables T, const float *__restrict__ q,
                                                float *__restrict__ tr) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M.E) return;
  const uint32_t E4 = uint32_t(M.E) * 4u;
  const rsrc_t rq = make_rsrc(q, 4u * N * N * E4), rt = make_rsrc(tr, 16u * N * E4);
  const uint32_t ve = uint32_t(e) * 4u;
  bool ex[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) ex[f] = face_exported(M.face[long(f) * M.E + e]);
  if (!(ex[0] || ex[1] || ex[2] || ex[3])) return;
  float Q[4][N][N];
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int j = 0; j < N; ++j)
#pragma unroll
      for (int i = 0; i < N; ++i) Q[v][j][i] = bload(rq, ve, ((v * N + j) * N + i) * E4);
#pragma unroll
  for (int p = 0; p < N; ++p) {
    float f0[4], f1[4], f2[4], f3[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      f0[v] = f1[v] = f2[v] = f3[v] = 0.f;
#pragma unroll
      for (int s = 0; s < N; ++s) {
        f0[v] += T.I[0][s] * Q[v][s][p];   // eta = 0, point p along xi
        f2[v] += T.I[N][s] * Q[v][s][p];   // eta = 1
        f1[v] += T.I[N][s] * Q[v][p][s];   // xi = 1, point p along eta
        f3[v] += T.I[0][s] * Q[v][p][s];   // xi = 0
      }
    }
    const uint32_t vo = (uint32_t(e) * N + p) * 16u, fs = uint32_t(M.E) * N * 16u;
    if (ex[0]) bstore4(f0, rt, vo, 0 * fs);
    if (ex[1]) bstore4(f1, rt, vo, 1 * fs);
    if (ex[2]) bstore4(f2, rt, vo, 2 * fs);
    if (ex[3]) bstore4(f3, rt, vo, 3 * fs);
  }
}

// ---------------------------------------------------------------------------
// the element residual, optionally fused with an SSP-RK stage update
//   rk = false:  out = dQ/dt
//   rk = true :  out = a qn + b (q + dt dQ/dt), exported face traces of out
//                -> trout
//
// A block owns EB = 64 consecutive elements and has N waves; lane l of
// wave w serves element (block * 64 + l).
//   row phase    (row j = w): interior xi-direction flux points (Xf_k, X_w),
//                then (once the block's state is in LDS) the faces xi = 0, 1
//                at point w; the xi part of the residual of row w -> LDS
//   column phase (column i = w): the same along eta with the faces eta = 0,
//                1 at point w, plus the row parts from LDS -> dQ/dt on
//                column w; RK update, column store, traces of faces eta = 0,
//                1 at point w
//   trace phase  (row w): traces of faces xi = 0, 1 at point w
// A neighbour in the same block is read from the block's LDS state, any
// other through the trace buffer.  LDS arrays are [var][j][i][lane]: every
// LDS access of a wave to its own elements touches 64 distinct banks.
// Global accesses of a wave are contiguous 256-byte rows.
// ---------------------------------------------------------------------------
template <int N, bool RK>
__global__ __launch_bounds__(64 * N) void k_stage(DevMesh M, OpTables T, Rotation R,
                                                  const float *q, const float *qn, float *out,
                                                  const float *trin, float *trout,
                                                  const float *mflux, float a, float b, float dt) {
  __shared__ float S[4][N][N][EB];     // state of the block's elements
  __shared__ float SR[4][N][N][EB];    // xi part of the residual, then the new state
  const float *Sf = &S[0][0][0][0];
  const int l = threadIdx.x & (EB - 1);
  // the wave index is uniform across the wave (blocks are 64 N lanes): say so,
  // so that offsets derived from it live in SGPRs
  const int w = __builtin_amdgcn_readfirstlane(int(threadIdx.x) / EB);
  const int e0 = blockIdx.x * EB + l;
  const bool valid = e0 < M.E;
  const int e = valid ? e0 : M.E - 1;
  const float gm1 = M.gamma - 1.0f;

  StageBufs B;
  B.E4 = uint32_t(M.E) * 4u;
  B.S4 = uint32_t(2 * M.K) * 4u;
  const uint32_t sbytes = 4u * N * N * B.E4, tbytes = 16u * N * B.E4;
  B.q = make_rsrc(q, sbytes);
  B.qn = make_rsrc(qn, RK ? sbytes : 0u);
  B.out = make_rsrc(out, sbytes);
  B.trin = make_rsrc(trin, tbytes);
  B.trout = make_rsrc(trout, RK ? tbytes : 0u);
  B.mflux = make_rsrc(mflux, 4u * N * B.S4);
  const uint32_t ve = uint32_t(e) * 4u;

  const long E = M.E;
  // ---- everything the element needs from memory, issued up front
  const uint32_t fw0 = M.face[0 * E + e], fw1 = M.face[1 * E + e];
  const uint32_t fw2 = M.face[2 * E + e], fw3 = M.face[3 * E + e];
  float qr[4][N];
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int i = 0; i < N; ++i) qr[v][i] = bload(B.q, ve, ((v * N + w) * N + i) * B.E4);
  const ElemGeo g = load_geo(M, e, R);
  float x0[4], x1[4], x2[4], x3[4];
  prefetch_face<N>(M, B, fw3, w, x3);   // row faces xi = 0, 1 at point w
  prefetch_face<N>(M, B, fw1, w, x1);
  prefetch_face<N>(M, B, fw0, w, x0);   // column faces eta = 0, 1 at point w
  prefetch_face<N>(M, B, fw2, w, x2);

  // ---- row phase
  {
    float res[4][N], t0[4], tN[4];
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int i = 0; i < N; ++i) {
        S[v][w][i][l] = qr[v][i];
        res[v][i] = 0.0f;
      }
#pragma unroll
    for (int k = 1; k < N; ++k) {
      float qf[4], f[4], nx, ny, vgn;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        float acc = 0.f;
#pragma unroll
        for (int i = 0; i < N; ++i) acc += T.I[k][i] * qr[v][i];
        qf[v] = acc;
      }
      metric_xi<N>(g, M, T, k, w, nx, ny, vgn);
      flux_n(qf, nx, ny, vgn, gm1, f);
#pragma unroll
      for (int i = 0; i < N; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) res[v][i] -= T.D[i][k] * f[v];
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      float s0 = 0.f, sN = 0.f;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        s0 += T.I[0][i] * qr[v][i];
        sN += T.I[N][i] * qr[v][i];
      }
      t0[v] = s0;
      tN[v] = sN;
    }
    __syncthreads();   // the block's state is in LDS
    {
      float f[4], nx, ny, vgn;
      metric_xi<N>(g, M, T, 0, w, nx, ny, vgn);       // face xi = 0: outward is -n
      common_flux<N>(M, T, Sf, fw3, w, t0, x3, -nx, -ny, -vgn, f);
#pragma unroll
      for (int i = 0; i < N; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) res[v][i] += T.D[i][0] * f[v];
      metric_xi<N>(g, M, T, N, w, nx, ny, vgn);       // face xi = 1: outward is +n
      common_flux<N>(M, T, Sf, fw1, w, tN, x1, nx, ny, vgn, f);
#pragma unroll
      for (int i = 0; i < N; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) res[v][i] -= T.D[i][N] * f[v];
    }
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int i = 0; i < N; ++i) SR[v][w][i][l] = res[v][i];
  }
  __syncthreads();

  // ---- column phase
  float qc[4][N], rc[4][N], qo[4][N];
  if (RK && a != 0.0f) {
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int j = 0; j < N; ++j) qo[v][j] = bload(B.qn, ve, ((v * N + j) * N + w) * B.E4);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int j = 0; j < N; ++j) {
      qc[v][j] = S[v][j][w][l];
      rc[v][j] = SR[v][j][w][l];
    }
#pragma unroll
  for (int k = 0; k <= N; ++k) {
    float qf[4], f[4], nx, ny, vgn;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      float acc = 0.f;
#pragma unroll
      for (int j = 0; j < N; ++j) acc += T.I[k][j] * qc[v][j];
      qf[v] = acc;
    }
    metric_eta<N>(g, M, T, k, w, nx, ny, vgn);
    if (k == 0) {
      common_flux<N>(M, T, Sf, fw0, w, qf, x0, -nx, -ny, -vgn, f);   // outward is -n
#pragma unroll
      for (int v = 0; v < 4; ++v) f[v] = -f[v];
    } else if (k == N) {
      common_flux<N>(M, T, Sf, fw2, w, qf, x2, nx, ny, vgn, f);
    } else {
      flux_n(qf, nx, ny, vgn, gm1, f);
    }
#pragma unroll
    for (int j = 0; j < N; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) rc[v][j] -= T.D[j][k] * f[v];
  }
  // dQ/dt = dQ~/dt / |J| on column w
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const float ij = inv_jacobian<N>(g, M, T, j, w);
#pragma unroll
    for (int v = 0; v < 4; ++v) rc[v][j] *= ij;
  }
  if (!RK) {
    if (valid) {
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int j = 0; j < N; ++j) bstore(rc[v][j], B.out, ve, ((v * N + j) * N + w) * B.E4);
    }
    return;
  }

  // ---- SSP-RK stage on column w: Q <- a Qn + b (Q + dt R); the new column
  // goes to SR (no other lane reads column w of SR after the column phase
  // has started)
  bool bad = false;
#pragma unroll
  for (int j = 0; j < N; ++j) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      float x = b * (qc[v][j] + dt * rc[v][j]);
      if (a != 0.0f) x += a * qo[v][j];
      qc[v][j] = x;
      SR[v][j][w][l] = x;
    }
    const float rho = qc[0][j];
    const float pr = gm1 * (qc[3][j] - 0.5f * (qc[1][j] * qc[1][j] + qc[2][j] * qc[2][j]) *
                                           __builtin_amdgcn_rcpf(rho));
    bad |= !(rho > 0.0f) || !(pr > 0.0f) || !isfinite(qc[1][j]) || !isfinite(qc[2][j]);
  }
  const bool ex0 = face_exported(fw0), ex2 = face_exported(fw2);
  const uint32_t tvo = (uint32_t(e) * N + uint32_t(w)) * 16u, tfs = uint32_t(M.E) * N * 16u;
  if (valid) {
    float f0[4], f2[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      f0[v] = f2[v] = 0.f;
#pragma unroll
      for (int j = 0; j < N; ++j) {
        bstore(qc[v][j], B.out, ve, ((v * N + j) * N + w) * B.E4);
        f0[v] += T.I[0][j] * qc[v][j];     // eta = 0 face, point w
        f2[v] += T.I[N][j] * qc[v][j];     // eta = 1 face, point w
      }
    }
    if (ex0) bstore4(f0, B.trout, tvo, 0 * tfs);
    if (ex2) bstore4(f2, B.trout, tvo, 2 * tfs);
    if (bad) M.flag[0] = 1;
  }
  __syncthreads();

  // ---- trace phase: faces xi = 0, 1 at point w from row w of the new state
  const bool ex1 = face_exported(fw1), ex3 = face_exported(fw3);
  if (valid && (ex1 || ex3)) {
    float f1[4], f3[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      f1[v] = f3[v] = 0.f;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const float x = SR[v][w][i][l];
        f1[v] += T.I[N][i] * x;
        f3[v] += T.I[0][i] * x;
      }
    }
    if (ex1) bstore4(f1, B.trout, tvo, 1 * tfs);
    if (ex3) bstore4(f3, B.trout, tvo, 3 * tfs);
  }
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
    for (int v = 0; v < 4; ++v) q[v][a] = double(tr[((long(f) * E + e) * N + pa) * 4 + v]);
  }
}

// One lane per interface face (L faces 0..K-1, R faces K..2K-1).  Each lane
// forms its face's two mortars: projects both sides' traces onto the mortar
// (eq. prjQ2), takes the Rusanov flux with the exact radial normal, scales
// it to flux per unit face parameter (R_s Delta), and projects back to its
// own face (eq. prjF2).  Output: outward common flux in the element's face
// parameter order, mflux[slot][point][var].
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
#pragma unroll
  for (int a = 0; a < N; ++a) {
    const int pa = flip ? N - 1 - a : a;
#pragma unroll
    for (int v = 0; v < 4; ++v) mflux[(long(t) * N + pa) * 4 + v] = float(sign * acc[v][a]);
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

constexpr int STAGE_BLOCK = 256;

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
  const int grid = (M.E + EB - 1) / EB;
  if (rk) {
    SSD_DISPATCH_N(M.N, hipLaunchKernelGGL((k_stage<NN, true>), dim3(grid), dim3(EB * NN), 0, s,
                                           M, T, rot, q, qn, out, trin, trout, mflux, a, b, dt));
  } else {
    SSD_DISPATCH_N(M.N, hipLaunchKernelGGL((k_stage<NN, false>), dim3(grid), dim3(EB * NN), 0, s,
                                           M, T, rot, q, qn, out, trin, trout, mflux, a, b, dt));
  }
  return hipGetLastError();
}

}  // namespace ssd

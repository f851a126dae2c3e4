// Device bodies of the SSD kernels for gfx950 (CDNA4): per-tile and
// per-chunk routines and the single-mesh __global__ wrappers, shared by the
// single-mesh launchers (ssd_kernels.hip) and the batched ones (ssd_batch.hip).
//
// Layout: per-cell arrays are cell-blocked (cb_index): blocks of 64
// consecutive elements, each stored plane after plane with one row of its
// elements per plane, so the wave that serves a block's 64 elements reads
// and writes contiguous 256-byte rows per (variable, point) and a block's
// state is one contiguous span.  Face traces (the solution interpolated to the
// element-boundary flux points) travel between blocks through a trace buffer
// laid out [face][element][point][var]: one lane moves the 4 variables of a
// point as one 16-byte access, and the N waves of a block together touch
// whole 16 N-byte face records.  Viscous gradient traces use the same layout
// with 8 values per point (x derivatives of the 4 variables, then y).
//
// Precision: state, traces and fluxes in FP32; element metrics and the
// sliding-interface projections in FP64.
#pragma once

#include "ssd_device.h"

namespace ssd {

// ---------------------------------------------------------------------------
// face traces of a state, for the faces some other block reads
// ---------------------------------------------------------------------------
template <int N>
__device__ __forceinline__ void traces_block(const DevMesh &M, const OpTables &T,
                                             const float *__restrict__ q, float *__restrict__ tr,
                                             int block) {
  const int e = block * TRACE_BLOCK + int(threadIdx.x);
  if (e >= M.E) return;
  const uint32_t E4 = uint32_t(M.E) * 4u;
  const rsrc_t rq = make_rsrc(q, 4u * N * N * E4), rt = make_rsrc(tr, 16u * N * E4);
  // cell-blocked state: plane 0 of cell e and the bytes of one plane row
  const uint32_t b = uint32_t(e) / EB;
  const uint32_t vq = (b * EB * 4u * N * N + (uint32_t(e) - b * EB)) * 4u;
  const uint32_t rowb = uint32_t(cb_rows(b, M.E)) * 4u;
  bool ex[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) ex[f] = face_exported(M.face[cb_index32(uint32_t(e), f, 4u, uint32_t(M.E))]);
  if (!(ex[0] || ex[1] || ex[2] || ex[3])) return;
  float Q[4][N][N];
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int j = 0; j < N; ++j)
#pragma unroll
      for (int i = 0; i < N; ++i) Q[v][j][i] = bload(rq, vq + ((v * N + j) * N + i) * rowb, 0u);
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

template <int N>
__global__ __launch_bounds__(TRACE_BLOCK) void k_traces(DevMesh M, OpTables T,
                                                        const float *__restrict__ q,
                                                        float *__restrict__ tr) {
  traces_block<N>(M, T, q, tr, blockIdx.x);
}

// Viscous inputs of the stage kernel (null on inviscid meshes).
struct ViscBufs {
  const float *G;       // grad Q at the SPs [(c*4+v)][j][i][E], c = 0 x, 1 y
  const float *gtr;     // gradient traces [face][E][point][8]
  const float *mvflux;  // viscous mortar flux [slot][point][4]
};

// Orders whose viscous stage passes gradient traces between the block's
// elements through LDS: the exchange array, [side][8][N][65] floats (16.25 KB
// at N = 4), keeps the stage at three blocks per compute unit.
template <int N>
__device__ constexpr bool grad_shared() {
  return N <= 4;
}

// An in-block face (the neighbour in the same block, across a face of the
// same direction with the same point order): the neighbour's gradient trace
// at point p comes from the same wave of the stage kernel (row phase: row
// p; column phase: column p), which leaves it in the block's exchange
// array just before it reads it.
template <int N>
__device__ __forceinline__ bool grad_in_block(uint32_t fw) {
  return grad_shared<N>() && face_inblock_of(fw);
}

// Lane stride of the gradient exchange array: one column more than the
// block's lanes, column EB holding zeros, so that a lane without an
// in-block neighbour adds zero by its address instead of by a select.
constexpr int XB = EB + 1;

// Faces whose gradient traces the gradient pass writes: sliding faces (the
// viscous mortar reads them) and the conforming faces without
// grad_in_block (both sides average the two).
template <int N>
__device__ __forceinline__ bool grad_exported(uint32_t fw) {
  const int k = face_kind_of(fw);
  if (k == SSD_FACE_SLIDING) return true;
  return (k == SSD_FACE_INTERIOR || k == SSD_FACE_PERIODIC) && !grad_in_block<N>(fw);
}

// Gradient traces at the two ends of a line of solution points (flux
// points 0 and N) into the exchange array at point p: g [8][N] along the
// line, X [side][8][N][XB].
template <int N>
__device__ __forceinline__ void share_traces(const OpTables &T, const float (&g)[8][N], float *X,
                                             int p, int lane) {
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    float s0 = 0.f, sN = 0.f;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      s0 += T.I[0][i] * g[c][i];
      sN += T.I[N][i] * g[c][i];
    }
    X[((0 * 8 + c) * N + p) * XB + lane] = s0;
    X[((1 * 8 + c) * N + p) * XB + lane] = sN;
  }
}

// Common viscous normal flux at one element-boundary flux point (BR1
// reading): F_vis(Q_c, mean of both gradients) . n on conforming faces,
// F_vis(Q_b, interior gradient) . n on isothermal walls and the far field,
// zero on slip walls, the mortar value on sliding faces.  qx: neighbour's
// state from common_flux; g: own gradient at the point [x0..x3, y0..y3].
// gbytes: the size of the trace buffer behind rgtr; X: the block's
// exchange array (grad_shared<N>()), else null.
template <int N>
__device__ __forceinline__ void common_visc(const DevMesh &M, const ViscParams &P, rsrc_t rgtr,
                                            uint32_t gbytes, rsrc_t rmv, const float *X,
                                            uint32_t fw, int p, const float qo[4],
                                            const float qx[4], const float x[4],
                                            const float g[8], const FPGeo &G, float fv[4]) {
  const int kind = face_kind_of(fw);
  if (kind == SSD_FACE_WALL_SLIP) {
#pragma unroll
    for (int v = 0; v < 4; ++v) fv[v] = 0.0f;
    return;
  }
  if (kind == SSD_FACE_SLIDING) {
    const f4 t = bload4(rmv, (uint32_t(face_idx_of(fw)) * N + uint32_t(p)) * 16u, 0u);
#pragma unroll
    for (int v = 0; v < 4; ++v) fv[v] = t.x[v];
    return;
  }
  float qc[4], gx[4], gy[4];
  common_solution(M, kind, qo, qx, x, G, qc);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    gx[v] = g[v];
    gy[v] = g[4 + v];
  }
  if (conforming(kind)) {
    // grad_in_block lanes point the loads past the end of the trace buffer
    // (zero, no memory access) and add the trace from the exchange array:
    // one load per lane, no branch, and either term exactly zero
    const bool inb = grad_in_block<N>(fw);
    const uint32_t nb = uint32_t(face_idx_of(fw)), nf = uint32_t(face_nf_of(fw));
    const uint32_t pp = face_rev_of(fw) ? uint32_t(N - 1 - p) : uint32_t(p);
    const uint32_t vo = inb ? gbytes : ((nf * uint32_t(M.E) + nb) * N + pp) * 32u;
    const f4 a = bload4(rgtr, vo, 0u), b = bload4(rgtr, vo + 16u, 0u);
    float gn[8];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      gn[v] = a.x[v];
      gn[4 + v] = b.x[v];
    }
    if (grad_shared<N>()) {
      // the neighbour's side of the array: xi = 1 / eta = 1 for faces 1, 2;
      // the zero column for the other lanes
      const int side = (nf == 1u || nf == 2u) ? 1 : 0;
      const float *xs = X + (side * 8 * N + p) * XB + (inb ? int(nb & uint32_t(EB - 1)) : EB);
#pragma unroll
      for (int c = 0; c < 8; ++c) gn[c] += xs[c * N * XB];
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      gx[v] = 0.5f * (gx[v] + gn[v]);
      gy[v] = 0.5f * (gy[v] + gn[4 + v]);
    }
  }
  visc_flux_n<float>(qc, gx, gy, G.nx, G.ny, P.mu, P.kT, fv);
}

// ---------------------------------------------------------------------------
// the element residual, optionally fused with an SSP Runge-Kutta stage
//   rk = false:  out = dQ/dt
//   rk = true :  out = qn + beta (q - qn) + gamma dt dQ/dt [+ add], the
//                Shu-Osher stage (1 - beta) qn + beta q + gamma dt dQ/dt
//                written around qn: the rounding then scales with the stage
//                increment, not with Q, and a steady state stays fixed
//                instead of drifting by an ulp per stage.  qn = null stands
//                for qn = q (first stage).  ADD: plus a precomputed increment
//                (the last SSPRK54 stage).  Exported face traces of out ->
//                trout.
//   visc:        adds the viscous fluxes, from the gradients of k_grad
//
// A block owns EB = 64 consecutive elements and has N waves; lane l of
// wave w serves element (block * 64 + l).
//   row phase    (row j = w): interior xi-direction flux points (Xf_k, X_w),
//                then (once the block's state is in LDS) the faces xi = 0, 1
//                at point w; the xi part of the residual of row w -> LDS
//   column phase (column i = w): the same along eta with the faces eta = 0,
//                1 at point w, plus the row parts from LDS -> dQ/dt on
//                column w; RK update into LDS, column store
//   pack phase   the face records some other block reads, computed from the
//                new state in LDS, one face per wave, whole records per
//                element
// An in-block neighbour's trace (face word bit: same block, same
// direction, same point order) comes from the exchange array the same wave
// filled with its own line's end traces (inviscid, N <= 4), or is
// interpolated from the block's LDS state; any other neighbour's comes
// through the trace buffer.  LDS arrays are [var][j][i][lane]: every LDS
// access of a wave to its own elements touches 64 distinct banks.  Global
// accesses of a wave are contiguous 256-byte rows.
// ---------------------------------------------------------------------------
//
// TPB tiles per block (batched stage): the block's waves form TPB groups of
// N, group g serving its own tile with its own LDS arrays; every group
// passes the same barriers.  A group with active = false (the block's last
// tiles past the end of the work table) is handed a valid tile, loads it,
// and stores nothing.
template <int N, bool RK, bool VISC, bool ADD, bool COMB = false, int TPB = 1>
__device__ __forceinline__ void stage_tile(const DevMesh &M, const OpTables &T, const Rotation &R,
                                           const float *q, const float *qn, float *out,
                                           const float *facein, float *trout, const ViscBufs &V,
                                           const RKCoef &C, int tile, bool active = true) {
  __shared__ float S_[TPB][4][N][N][EB];    // state of the group's elements
  __shared__ float SR_[TPB][4][N][N][EB];   // xi part of the residual, then the new state
  // viscous, grad_shared<N>(): the gradient traces of the current phase's
  // faces, [side][8][point][lane, then a zero column]; point w is written
  // and read by wave w alone (in order within the wave), so it needs no
  // barrier
  constexpr bool GS = VISC && grad_shared<N>();
  __shared__ float X_[TPB][GS ? 2 * 8 * N * XB : 1];
  // inviscid, trace_shared<N>(): the solution traces of the current
  // phase's faces, [side][4][point][lane], point w again wave w's alone
  constexpr bool SX = !VISC && trace_shared<N>();
  __shared__ float XS_[TPB][SX ? 2 * 4 * N * EB : 1];
  // the wave index and the group are uniform across the wave: say so, so
  // that offsets derived from them live in SGPRs
  const int grp = TPB > 1 ? __builtin_amdgcn_readfirstlane(int(threadIdx.x) / (EB * N)) : 0;
  float(&S)[4][N][N][EB] = S_[grp];
  float(&SR)[4][N][N][EB] = SR_[grp];
  const float *Sf = &S[0][0][0][0];
  float *X = GS ? X_[grp] : nullptr;
  float *XS = SX ? XS_[grp] : nullptr;
  const int l = threadIdx.x & (EB - 1);
  const int w = __builtin_amdgcn_readfirstlane((int(threadIdx.x) / EB) % N);
  const int e0 = tile * EB + l;
  const bool valid = active && e0 < M.E;
  const int e = valid ? e0 : M.E - 1;
  const float gm1 = M.gamma - 1.0f;
  const uint32_t E4 = uint32_t(M.E) * 4u;
  const uint32_t sbytes = 4u * N * N * E4, tbytes = 16u * N * E4;
  const uint32_t mbytes = uint32_t(2 * M.K) * N * 16u;
  const rsrc_t rq = make_rsrc(q, sbytes);
  const rsrc_t rqn = make_rsrc(qn, RK ? sbytes : 0u);
  const rsrc_t rout = make_rsrc(out, sbytes);
  // face data of q: traces, then the mortar flux records
  const uint32_t fbytes = tbytes + mbytes;
  const rsrc_t rtin = make_rsrc(facein, fbytes);
  const rsrc_t rtout = make_rsrc(trout, RK ? tbytes : 0u);
  const rsrc_t rG = make_rsrc(V.G, VISC ? 2u * sbytes : 0u);
  const rsrc_t rgtr = make_rsrc(V.gtr, VISC ? 2u * tbytes : 0u);
  const rsrc_t rmv = make_rsrc(V.mvflux, VISC ? mbytes : 0u);
  const rsrc_t rcomb = make_rsrc(C.comb, (RK && COMB) ? sbytes : 0u);
  const ViscParams P = visc_params(M);
  // cell-blocked state and gradient arrays: plane 0 of the lane's cell, and
  // the bytes of one plane row of this block (uniform)
  const uint32_t nbt = uint32_t(__builtin_amdgcn_readfirstlane(int(cb_rows(tile, M.E))));
  const uint32_t lc = valid ? uint32_t(l) : nbt - 1u;
  const uint32_t vs = (uint32_t(tile) * (EB * 4u * N * N) + lc) * 4u;
  const uint32_t vg = (uint32_t(tile) * (EB * 8u * N * N) + lc) * 4u;
  const uint32_t rowb = nbt * 4u;
  const long E = M.E;

  // ---- everything the element needs from memory, issued up front.  The
  // state arrays (Q_k, Qn and the stage's output, and the RK increments)
  // are read or written once per launch and are far larger than the
  // caches: they take the non-temporal policy, so that they do not push out
  // the face words, geometry and face traces, which every stage reads again,
  // nor (viscous) the gradient rows the column phase reads a second time.
  const uint32_t fw0 = M.face[cb_index32(uint32_t(e), 0u, 4u, uint32_t(E))];
  const uint32_t fw1 = M.face[cb_index32(uint32_t(e), 1u, 4u, uint32_t(E))];
  const uint32_t fw2 = M.face[cb_index32(uint32_t(e), 2u, 4u, uint32_t(E))];
  const uint32_t fw3 = M.face[cb_index32(uint32_t(e), 3u, 4u, uint32_t(E))];
  float qr[4][N];
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int i = 0; i < N; ++i) qr[v][i] = bload_nt(rq, vs, ((v * N + w) * N + i) * rowb);
  const ElemGeo g = load_geo(M, e, R);
  float x0[4], x1[4], x2[4], x3[4];
  prefetch_face<N>(M, rtin, fbytes, tbytes, uint32_t(M.E), fw3, w, x3);   // row faces xi = 0, 1 at point w
  prefetch_face<N>(M, rtin, fbytes, tbytes, uint32_t(M.E), fw1, w, x1);
  if (!VISC) {   // column faces eta = 0, 1 (viscous stages: at the column phase)
    prefetch_face<N>(M, rtin, fbytes, tbytes, uint32_t(M.E), fw0, w, x0);
    prefetch_face<N>(M, rtin, fbytes, tbytes, uint32_t(M.E), fw2, w, x2);
  }
  float qo[4][N];   // column w of Qn (RK stages after the first)
  const bool with_qn = RK && qn != nullptr;
  if (with_qn && !VISC) {   // viscous stages load these just before the update
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int j = 0; j < N; ++j) qo[v][j] = bload_nt(rqn, vs, ((v * N + j) * N + w) * rowb);
  }
  float qa[4][N];   // column w of the added increment (ADD)
  if (RK && ADD) {
    const rsrc_t radd = make_rsrc(C.add, sbytes);
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int j = 0; j < N; ++j) qa[v][j] = bload_nt(radd, vs, ((v * N + j) * N + w) * rowb);
  }

  // ---- row phase
  {
    const LineGeo Lr = line_xi(g, float(T.X[w]));   // bilinear-cell metrics along row w
    float res[4][N], t0[4], tN[4];
    float gr[8][N];   // gradient on row w
    if (VISC) {
#pragma unroll
      for (int c = 0; c < 8; ++c)
#pragma unroll
        for (int i = 0; i < N; ++i) gr[c][i] = bload(rG, vg, ((c * N + w) * N + i) * rowb);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int i = 0; i < N; ++i) {
        S[v][w][i][l] = qr[v][i];
        res[v][i] = 0.0f;
      }
#pragma unroll
    for (int k = 1; k < N; ++k) {
      float qf[4], f[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        float acc = 0.f;
#pragma unroll
        for (int i = 0; i < N; ++i) acc += T.I[k][i] * qr[v][i];
        qf[v] = acc;
      }
      const FPGeo G = metric_xi<N>(g, Lr, M, T, k, w);
      flux_n(qf, G.nx, G.ny, G.vgn, gm1, f);
      if (VISC) {
        float gf[8], fv[4];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          float acc = 0.f;
#pragma unroll
          for (int i = 0; i < N; ++i) acc += T.I[k][i] * gr[c][i];
          gf[c] = acc;
        }
        visc_flux_n<float>(qf, gf, gf + 4, G.nx, G.ny, P.mu, P.kT, fv);
#pragma unroll
        for (int v = 0; v < 4; ++v) f[v] += fv[v];
      }
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
    if (GS) {
      share_traces<N>(T, gr, X, w, l);
      // the zero column, 16 N entries, before the barrier below and never
      // written again
      if (w == 0 && l < 16 * N) X[l * XB + EB] = 0.f;
    }
    if (SX) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        XS[(v * N + w) * EB + l] = t0[v];
        XS[((4 + v) * N + w) * EB + l] = tN[v];
      }
    }
    __syncthreads();   // the block's state is in LDS
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const int k = side ? N : 0;
      const float sg = side ? 1.0f : -1.0f;   // outward normal of face xi = 1 / xi = 0
      const uint32_t fw = side ? fw1 : fw3;
      FPGeo G = metric_xi<N>(g, Lr, M, T, k, w);
      G.nx *= sg;
      G.ny *= sg;
      G.vgn *= sg;
      float f[4], qx[4];
      neighbor_state_x<N, SX>(T, Sf, XS, fw, w, side ? x1 : x3, qx);
      common_flux(M, fw, side ? tN : t0, qx, side ? x1 : x3, G, f);
      if (VISC) {
        float gf[8], fv[4];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          float acc = 0.f;
#pragma unroll
          for (int i = 0; i < N; ++i) acc += T.I[k][i] * gr[c][i];
          gf[c] = acc;
        }
        common_visc<N>(M, P, rgtr, 2u * tbytes, rmv, X, fw, w, side ? tN : t0, qx,
                       side ? x1 : x3, gf, G, fv);
#pragma unroll
        for (int v = 0; v < 4; ++v) f[v] += fv[v];
      }
#pragma unroll
      for (int i = 0; i < N; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) res[v][i] -= T.D[i][k] * (sg * f[v]);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int i = 0; i < N; ++i) SR[v][w][i][l] = res[v][i];
  }
  __syncthreads();

  // ---- column phase
  float qc[4][N], rc[4][N];
  if (VISC) {
    prefetch_face<N>(M, rtin, fbytes, tbytes, uint32_t(M.E), fw0, w, x0);
    prefetch_face<N>(M, rtin, fbytes, tbytes, uint32_t(M.E), fw2, w, x2);
  }
  {
    const LineGeo Lc = line_eta(g, float(T.X[w]));  // bilinear-cell metrics along column w
    float gc[8][N];   // gradient on column w (its last read: non-temporal)
    if (VISC) {
#pragma unroll
      for (int c = 0; c < 8; ++c)
#pragma unroll
        for (int j = 0; j < N; ++j) gc[c][j] = bload_nt(rG, vg, ((c * N + j) * N + w) * rowb);
    }
    if (GS) {
      share_traces<N>(T, gc, X, w, l);
      // keeps the scheduler from hoisting the column loop's work above the
      // exchange (registers: the viscous N = 4 stage stays at 3 waves/SIMD)
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int j = 0; j < N; ++j) {
        qc[v][j] = S[v][j][w][l];
        rc[v][j] = SR[v][j][w][l];
      }
    if (SX) {   // this column's traces at eta = 0, 1
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        float s0 = 0.f, sN = 0.f;
#pragma unroll
        for (int j = 0; j < N; ++j) {
          s0 += T.I[0][j] * qc[v][j];
          sN += T.I[N][j] * qc[v][j];
        }
        XS[(v * N + w) * EB + l] = s0;
        XS[((4 + v) * N + w) * EB + l] = sN;
      }
    }
    // viscous stages take the interior flux points first and the two faces
    // last (measured 1.5 % faster at N = 4)
#pragma unroll
    for (int kk = 0; kk <= N; ++kk) {
      const int k = !VISC ? kk : kk < N - 1 ? kk + 1 : kk == N - 1 ? 0 : N;
      float qf[4], f[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        float acc = 0.f;
#pragma unroll
        for (int j = 0; j < N; ++j) acc += T.I[k][j] * qc[v][j];
        qf[v] = acc;
      }
      FPGeo G = metric_eta<N>(g, Lc, M, T, k, w);
      float gf[8];
      if (VISC) {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          float acc = 0.f;
#pragma unroll
          for (int j = 0; j < N; ++j) acc += T.I[k][j] * gc[c][j];
          gf[c] = acc;
        }
      }
      if (k == 0 || k == N) {
        const float sg = k == 0 ? -1.0f : 1.0f;   // outward normal of face eta = 0 / eta = 1
        const uint32_t fw = k == 0 ? fw0 : fw2;
        G.nx *= sg;
        G.ny *= sg;
        G.vgn *= sg;
        float qx[4];
        neighbor_state_x<N, SX>(T, Sf, XS, fw, w, k == 0 ? x0 : x2, qx);
        common_flux(M, fw, qf, qx, k == 0 ? x0 : x2, G, f);
        if (VISC) {
          float fv[4];
          common_visc<N>(M, P, rgtr, 2u * tbytes, rmv, X, fw, w, qf, qx,
                         k == 0 ? x0 : x2, gf, G, fv);
#pragma unroll
          for (int v = 0; v < 4; ++v) f[v] += fv[v];
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) f[v] *= sg;
      } else {
        flux_n(qf, G.nx, G.ny, G.vgn, gm1, f);
        if (VISC) {
          float fv[4];
          visc_flux_n<float>(qf, gf, gf + 4, G.nx, G.ny, P.mu, P.kT, fv);
#pragma unroll
          for (int v = 0; v < 4; ++v) f[v] += fv[v];
        }
      }
#pragma unroll
      for (int j = 0; j < N; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) rc[v][j] -= T.D[j][k] * f[v];
    }
  }
  // dQ/dt = dQ~/dt / |J| on column w
  float ij[N];
#pragma unroll
  for (int j = 0; j < N; ++j) ij[j] = inv_jacobian<N>(g, M, T, j, w);
  if (!RK) {
    if (valid) {
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int j = 0; j < N; ++j)
          bstore_nt(rc[v][j] * ij[j], rout, vs, ((v * N + j) * N + w) * rowb);
    }
    return;
  }

  // ---- SSP-RK stage on column w: Q <- Qn + beta (Q - Qn) + gamma dt R
  // [+ add_scale add]; the new column goes to SR (no other lane reads column w of SR
  // after the column phase has started)
  if (VISC && with_qn) {   // viscous stages: Qn only now, to keep the column phase's registers down
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int j = 0; j < N; ++j) qo[v][j] = bload_nt(rqn, vs, ((v * N + j) * N + w) * rowb);
  }
  float u2[4][N];   // (COMB) column w of U2, loaded late for the same reason
  if (COMB) {
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int j = 0; j < N; ++j) u2[v][j] = bload_nt(rcomb, vs, ((v * N + j) * N + w) * rowb);
  }
  // the new value x of variable v at point j: the added increment, the
  // SSPRK54 combination (stages with Qn only), then the state
  auto commit = [&](int v, int j, float x, bool qn_stage) {
    if (ADD) x += C.add_scale * qa[v][j];
    if (COMB && qn_stage)
      u2[v][j] = C.cw2 * (u2[v][j] - qo[v][j]) + C.cw3 * (qc[v][j] - qo[v][j]) +
                 C.cw4 * (x - qo[v][j]);
    qc[v][j] = x;
    SR[v][j][w][l] = x;
  };
  // a uniform branch, not a per-value select, so that a stage computes
  // only its own form of the update
  if (with_qn) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const float gdt = C.gamma * C.dt * ij[j];
#pragma unroll
      for (int v = 0; v < 4; ++v)
        commit(v, j, qo[v][j] + (C.beta * (qc[v][j] - qo[v][j]) + gdt * rc[v][j]), true);
    }
  } else {
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const float gdt = C.gamma * C.dt * ij[j];
#pragma unroll
      for (int v = 0; v < 4; ++v) commit(v, j, qc[v][j] + gdt * rc[v][j], false);
    }
  }
  bool bad = false;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    // rho > 0 and p > 0, i.e. 2 rho E > |m|^2; false for any non-finite value
    const float rho = qc[0][j];
    bad |= !(rho > 0.0f) ||
           !(2.0f * rho * qc[3][j] > qc[1][j] * qc[1][j] + qc[2][j] * qc[2][j]);
  }
  if (valid) {
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int j = 0; j < N; ++j) bstore_nt(qc[v][j], rout, vs, ((v * N + j) * N + w) * rowb);
    if (COMB) {
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int j = 0; j < N; ++j) bstore_nt(u2[v][j], rcomb, vs, ((v * N + j) * N + w) * rowb);
    }
    if (bad) M.flag[0] = 1;
  }
  // lanes whose face f is read by another block (every wave holds the
  // same 64 elements, so every wave forms the same masks)
  const uint64_t xm[4] = {__builtin_amdgcn_ballot_w64(valid && face_exported(fw0)),
                          __builtin_amdgcn_ballot_w64(valid && face_exported(fw1)),
                          __builtin_amdgcn_ballot_w64(valid && face_exported(fw2)),
                          __builtin_amdgcn_ballot_w64(valid && face_exported(fw3))};
  __syncthreads();   // the new state of the whole block is in SR

  // ---- pack phase: wave w writes the face records of faces f = w, w + N,
  // ...  Lane k of a chunk takes point k % N of the (k / N)-th listed
  // element, so the N lanes of an element write its whole 16 N-byte record
  // and one store instruction covers the records of 64 / N elements:
  // consecutive exporting elements give one contiguous span.
  constexpr int EPC = EB / N;   // elements per chunk
  const uint32_t tile0 = uint32_t(tile) * EB;
  for (int f = w; f < 4; f += N) {
    const uint64_t m = xm[f];
    const int cnt = __builtin_popcountll(m);
    // the list of exporting lanes in lane order, one entry per lane: a full
    // permutation pushes exporter l to lane rank(l) and every other lane
    // behind them, so lane k < cnt holds the k-th exporting lane
    const bool ex = (m >> l) & 1u;
    const int slot = ex ? lane_rank(m) : cnt + lane_rank(~m);
    const int listed = __builtin_amdgcn_ds_permute(slot * 4, l);
    for (int c0 = 0; c0 < cnt; c0 += EPC) {
      const int j = c0 + l / N, p = l % N;
      // all lanes take part in the pull; j < 64 always (c0 < cnt <= 64 and
      // l / N < EPC), lanes with j >= cnt discard what they read
      const int src = __builtin_amdgcn_ds_bpermute(min(j, EB - 1) * 4, listed);
      if (l < EPC * N && j < cnt) {
        float tv[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          float acc = 0.f;
          if (f == 0 || f == 2) {   // eta = 0 / eta = 1 at point p along xi
            const float *I = T.I[f == 0 ? 0 : N];
#pragma unroll
            for (int jj = 0; jj < N; ++jj) acc += I[jj] * SR[v][jj][p][src];
          } else {                  // xi = 1 / xi = 0 at point p along eta
            const float *I = T.I[f == 3 ? 0 : N];
#pragma unroll
            for (int i = 0; i < N; ++i) acc += I[i] * SR[v][p][i][src];
          }
          tv[v] = acc;
        }
        bstore4(tv, rtout, ((uint32_t(f) * uint32_t(M.E) + tile0 + uint32_t(src)) * N + p) * 16u,
                0u);
      }
    }
  }
}

// The plain inviscid stage at N <= 4 is held to 128 VGPRs, 4 waves per SIMD
// (the compiler otherwise settles one or two registers above, at 3).
template <int N, bool RK, bool VISC, bool ADD, bool COMB>
constexpr int stage_waves_per_eu() {
  return (!VISC && !ADD && !COMB && N <= 4) ? 4 : 1;
}

template <int N, bool RK, bool VISC, bool ADD, bool COMB = false>
__global__ __launch_bounds__(64 * N)
__attribute__((amdgpu_waves_per_eu(stage_waves_per_eu<N, RK, VISC, ADD, COMB>()))) void k_stage(
    DevMesh M, OpTables T, Rotation R, const float *q, const float *qn, float *out,
    const float *facein, float *trout, ViscBufs V, RKCoef C) {
  const int b = int(blockIdx.x);
  const int tile = !C.reverse ? b : b < C.lead ? b : int(gridDim.x) - 1 - (b - C.lead);
  stage_tile<N, RK, VISC, ADD, COMB>(M, T, R, q, qn, out, facein, trout, V, C, tile);
}

// ---------------------------------------------------------------------------
// viscous gradient pass (Sec. 3.1, BR1 reading)
//   Q_xi and Q_eta at the SPs are the derivatives of the degree-N
//   polynomials through the solution interpolated to the interior flux
//   points and the common solution at the element's faces (eqs. Ft, Gt
//   applied to Q); grad Q follows by the chain rule with the SP metrics.
// Outputs: grad Q at the SPs, G [(c*4+v)][j][i][E], stored with the
// non-temporal policy (the stage reads it once per phase, after other
// traffic); gradient traces, gtr [face][E][point][8], of the faces
// grad_exported names.
// Same block and wave organisation as k_stage.
// ---------------------------------------------------------------------------
template <int N>
__device__ __forceinline__ void grad_tile(const DevMesh &M, const OpTables &T, const Rotation &R,
                                          const float *q, const float *facein, float *Gout,
                                          float *gtr, int tile) {
  // LDS: the state and Q_xi while the derivatives are formed, then the
  // gradient of the whole block
  __shared__ float L[8][N][N][EB];
  float(*S)[N][N][EB] = L;        // [var][j][i][lane]
  float(*QX)[N][N][EB] = L + 4;   // Q_xi
  const float *Sf = &L[0][0][0][0];
  const int l = threadIdx.x & (EB - 1);
  const int w = __builtin_amdgcn_readfirstlane(int(threadIdx.x) / EB);
  const int e0 = tile * EB + l;
  const bool valid = e0 < M.E;
  const int e = valid ? e0 : M.E - 1;
  const uint32_t E4 = uint32_t(M.E) * 4u;
  const uint32_t sbytes = 4u * N * N * E4, tbytes = 16u * N * E4;
  const rsrc_t rq = make_rsrc(q, sbytes);
  // face data of q: traces, mortar flux records, then the mortar common
  // solution records read here
  const uint32_t mbytes = uint32_t(2 * M.K) * N * 16u;
  const uint32_t fbytes = tbytes + 2u * mbytes;
  const rsrc_t rtin = make_rsrc(facein, fbytes);
  const rsrc_t rG = make_rsrc(Gout, 2u * sbytes);
  const rsrc_t rgtr = make_rsrc(gtr, 2u * tbytes);
  // cell-blocked state and gradient arrays: plane 0 of the lane's cell, and
  // the bytes of one plane row of this block (uniform)
  const uint32_t nbt = uint32_t(__builtin_amdgcn_readfirstlane(int(cb_rows(tile, M.E))));
  const uint32_t lc = valid ? uint32_t(l) : nbt - 1u;
  const uint32_t vs = (uint32_t(tile) * (EB * 4u * N * N) + lc) * 4u;
  const uint32_t vg = (uint32_t(tile) * (EB * 8u * N * N) + lc) * 4u;
  const uint32_t rowb = nbt * 4u;
  const long E = M.E;

  const uint32_t fw0 = M.face[cb_index32(uint32_t(e), 0u, 4u, uint32_t(E))];
  const uint32_t fw1 = M.face[cb_index32(uint32_t(e), 1u, 4u, uint32_t(E))];
  const uint32_t fw2 = M.face[cb_index32(uint32_t(e), 2u, 4u, uint32_t(E))];
  const uint32_t fw3 = M.face[cb_index32(uint32_t(e), 3u, 4u, uint32_t(E))];
  float qr[4][N];
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int i = 0; i < N; ++i) qr[v][i] = bload(rq, vs, ((v * N + w) * N + i) * rowb);
  const ElemGeo g = load_geo(M, e, R);
  float x0[4], x1[4], x2[4], x3[4];
  prefetch_face<N>(M, rtin, fbytes, tbytes + mbytes, uint32_t(M.E), fw3, w, x3);
  prefetch_face<N>(M, rtin, fbytes, tbytes + mbytes, uint32_t(M.E), fw1, w, x1);
  prefetch_face<N>(M, rtin, fbytes, tbytes + mbytes, uint32_t(M.E), fw0, w, x0);
  prefetch_face<N>(M, rtin, fbytes, tbytes + mbytes, uint32_t(M.E), fw2, w, x2);
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int i = 0; i < N; ++i) S[v][w][i][l] = qr[v][i];
  __syncthreads();   // the block's state is in LDS

  // common solution at point p of a face with outward normal sign sg
  auto face_common = [&](uint32_t fw, bool xi_face, int k, float sg, const float qo[4],
                         const float x[4], float qcm[4]) {
    FPGeo G = xi_face ? metric_xi<N>(g, line_xi(g, float(T.X[w])), M, T, k, w)
                      : metric_eta<N>(g, line_eta(g, float(T.X[w])), M, T, k, w);
    G.nx *= sg;
    G.ny *= sg;
    G.vgn *= sg;
    float qx[4];
    const int kind = face_kind_of(fw);
    neighbor_state<N>(T, Sf, fw, w, x, qx);
    common_solution(M, kind, qo, qx, x, G, qcm);
  };

  // ---- row w: Q_xi
  {
    float qs[4][N + 1];
#pragma unroll
    for (int k = 0; k <= N; ++k)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        float acc = 0.f;
#pragma unroll
        for (int i = 0; i < N; ++i) acc += T.I[k][i] * qr[v][i];
        qs[v][k] = acc;
      }
    float c0[4], cN[4], o0[4], oN[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      o0[v] = qs[v][0];
      oN[v] = qs[v][N];
    }
    face_common(fw3, true, 0, -1.0f, o0, x3, c0);
    face_common(fw1, true, N, 1.0f, oN, x1, cN);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      qs[v][0] = c0[v];
      qs[v][N] = cN[v];
    }
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k <= N; ++k) acc += T.D[i][k] * qs[v][k];
        QX[v][w][i][l] = acc;
      }
  }

  // ---- column w: Q_eta
  float qe[4][N];
  {
    float qcol[4][N], qs[4][N + 1];
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int j = 0; j < N; ++j) qcol[v][j] = S[v][j][w][l];
#pragma unroll
    for (int k = 0; k <= N; ++k)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        float acc = 0.f;
#pragma unroll
        for (int j = 0; j < N; ++j) acc += T.I[k][j] * qcol[v][j];
        qs[v][k] = acc;
      }
    float c0[4], cN[4], o0[4], oN[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      o0[v] = qs[v][0];
      oN[v] = qs[v][N];
    }
    face_common(fw0, false, 0, -1.0f, o0, x0, c0);
    face_common(fw2, false, N, 1.0f, oN, x2, cN);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      qs[v][0] = c0[v];
      qs[v][N] = cN[v];
    }
#pragma unroll
    for (int j = 0; j < N; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k <= N; ++k) acc += T.D[j][k] * qs[v][k];
        qe[v][j] = acc;
      }
  }
  __syncthreads();   // Q_xi of every row is in LDS

  // ---- grad Q on column w:  Q_x = (y_eta Q_xi - y_xi Q_eta) / |J|,
  //                           Q_y = (x_xi Q_eta - x_eta Q_xi) / |J|
  float gcol[8][N];
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const SPGeo sp = metric_sp<N>(g, M, T, j, w);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const float qxi = QX[v][j][w][l];
      gcol[v][j] = (sp.ye * qxi - sp.yx * qe[v][j]) * sp.ij;
      gcol[4 + v][j] = (sp.xx * qe[v][j] - sp.xe * qxi) * sp.ij;
    }
  }
  const uint32_t gvo = (uint32_t(e) * N + uint32_t(w)) * 32u, gfs = uint32_t(M.E) * N * 32u;
  if (valid) {
    float f0[8], f2[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      f0[c] = f2[c] = 0.f;
#pragma unroll
      for (int j = 0; j < N; ++j) {
        bstore_nt(gcol[c][j], rG, vg, ((c * N + j) * N + w) * rowb);
        f0[c] += T.I[0][j] * gcol[c][j];
        f2[c] += T.I[N][j] * gcol[c][j];
      }
    }
    if (grad_exported<N>(fw0)) {
      bstore4(f0, rgtr, gvo, 0 * gfs);
      bstore4(f0 + 4, rgtr, gvo + 16u, 0 * gfs);
    }
    if (grad_exported<N>(fw2)) {
      bstore4(f2, rgtr, gvo, 2 * gfs);
      bstore4(f2 + 4, rgtr, gvo + 16u, 2 * gfs);
    }
  }
  __syncthreads();   // every wave has read its column of Q_xi: L is free
#pragma unroll
  for (int c = 0; c < 8; ++c)
#pragma unroll
    for (int j = 0; j < N; ++j) L[c][j][w][l] = gcol[c][j];
  __syncthreads();

  // ---- gradient traces of faces xi = 0, 1 at point w from row w
  const bool gx1 = grad_exported<N>(fw1), gx3 = grad_exported<N>(fw3);
  if (valid && (gx1 || gx3)) {
    float f1[8], f3[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      f1[c] = f3[c] = 0.f;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const float x = L[c][w][i][l];
        f1[c] += T.I[N][i] * x;
        f3[c] += T.I[0][i] * x;
      }
    }
    if (gx1) {
      bstore4(f1, rgtr, gvo, 1 * gfs);
      bstore4(f1 + 4, rgtr, gvo + 16u, 1 * gfs);
    }
    if (gx3) {
      bstore4(f3, rgtr, gvo, 3 * gfs);
      bstore4(f3 + 4, rgtr, gvo + 16u, 3 * gfs);
    }
  }
}

template <int N>
__global__ __launch_bounds__(64 * N) void k_grad(DevMesh M, OpTables T, Rotation R,
                                                 const float *q, const float *facein, float *Gout,
                                                 float *gtr, int reverse) {
  const int tile = reverse ? int(gridDim.x) - 1 - int(blockIdx.x) : int(blockIdx.x);
  grad_tile<N>(M, T, R, q, facein, Gout, gtr, tile);
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

// Placement (m, delta) of the interface faces for the rotor angle and the 8
// projection matrices, computed by the calling workgroup into `ms` (LDS).
// A_k(i,j) = int_0^1 h_i(z) h_j(o_k + s_k z) dz by N-point Gauss-Legendre
// quadrature (exact: degree 2N-2); P_fwd = M^-1 A (eq. prjQ2), P_back =
// s M^-1 A^T (eq. prjF2).
template <int N>
__device__ void build_mortar(const DevMesh &M, const MortarTables &MT, double theta,
                             MortarState &ms, double (&A)[4][N][N]) {
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
    ms.o[0] = 0.0;     ms.s[0] = 1.0 - d;   // L face, first mortar
    ms.o[1] = 1.0 - d; ms.s[1] = d;         // L face, second mortar
    ms.o[2] = d;       ms.s[2] = 1.0 - d;   // R face, first mortar
    ms.o[3] = 0.0;     ms.s[3] = d;         // R face, second mortar
    ms.m = int(mm);
    ms.delta = d;
    ms.thL = thL;
    ms.thR = thR;
    ms.valid = 1;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < 4 * N * N; idx += blockDim.x) {
    const int k = idx / (N * N), i = (idx / N) % N, j = idx % N;
    double acc = 0.0;
    for (int q = 0; q < N; ++q)
      acc += MT.wq[q] * MT.hq[q][i] * lagrange_d(MT, N, j, ms.o[k] + ms.s[k] * MT.zq[q]);
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
    ms.Pf[k][i][j] = f;
    ms.Pb[k][i][j] = ms.s[k] * bk;
  }
  __syncthreads();
}

// Copy of a mortar state from LDS to device memory by the workgroup.
__device__ __forceinline__ void store_mortar(const MortarState &src, MortarState *dst) {
  static_assert(sizeof(MortarState) % 8 == 0, "mortar state is copied as 8-byte words");
  const uint64_t *a = reinterpret_cast<const uint64_t *>(&src);
  uint64_t *b = reinterpret_cast<uint64_t *>(dst);
  for (int i = threadIdx.x; i < int(sizeof(MortarState) / 8); i += blockDim.x) b[i] = a[i];
}

// Mortar rebuild on its own (one workgroup), for the residual entry point.
template <int N>
__global__ __launch_bounds__(64) void k_rebuild(DevMesh M, MortarTables MT, double theta,
                                                MortarState *__restrict__ ms) {
  __shared__ MortarState S;
  __shared__ double A[4][N][N];
  build_mortar<N>(M, MT, theta, S, A);
  store_mortar(S, ms);
}

// C values per point of ring slot `slot` in the face's canonical
// (counter-clockwise) point order, from a [face][E][point][C] trace array.
template <int N, int C>
__device__ __forceinline__ void load_canon(const DevMesh &M, const float *__restrict__ tr, int slot,
                                           double q[C][N]) {
  const long E = M.E;
  const int e = M.ring_e[slot], f = M.ring_f[slot], flip = M.ring_flip[slot];
#pragma unroll
  for (int a = 0; a < N; ++a) {
    const int pa = flip ? N - 1 - a : a;
#pragma unroll
    for (int v = 0; v < C; ++v) q[v][a] = double(tr[((long(f) * E + e) * N + pa) * C + v]);
  }
}

// Sliding interface, inviscid: N lanes per interface face (L faces 0..K-1,
// R faces K..2K-1), lane a for point a.  Each workgroup first rebuilds the
// placement and projections for the rotor angle (block 0 also stores them
// for the viscous mortar).  For each of its face's two mortars a lane
// projects both sides' traces to mortar point a (eq. prjQ2), takes the
// Rusanov flux with the exact radial normal there, scaled to flux per unit
// face parameter (R_s Delta), and shares it through LDS; then it projects
// the mortar fluxes back to its own face point (eq. prjF2).  Output: outward
// common flux in the element's face parameter order, mflux[slot][point][var].
// With VISC also the common solution on the face for the gradient pass: the
// mean of the two sides' projections on each mortar, projected back
// (Sec. 3.2), mqc[slot][point][var].

template <int N, bool VISC>
__device__ __forceinline__ void mortar_chunk(const DevMesh &M, const OpTables &T,
                                             const MortarTables &MT, double theta,
                                             MortarState *ms_out, const float *__restrict__ tr,
                                             float *__restrict__ mflux, float *__restrict__ mqc,
                                             int chunk) {
  constexpr int FPB = MORTAR_BLOCK / N;   // faces per workgroup
  __shared__ MortarState S;
  __shared__ double A[4][N][N];
  __shared__ double FM[FPB][2][N][4];     // mortar fluxes at the mortar points
  __shared__ double QM[VISC ? FPB : 1][2][N][4];
  build_mortar<N>(M, MT, theta, S, A);
  if (chunk == 0) store_mortar(S, ms_out);
  const int K = M.K;
  const int fl = threadIdx.x / N, a = threadIdx.x % N;
  const int t = chunk * FPB + fl;
  const bool act = fl < FPB && t < 2 * K;
  const bool right = t >= K;
  const int j = right ? t - K : t;
  const int m = S.m;
  if (act) {
    const double sc = M.Rs * M.dphi;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int jl = right ? ((j - m - k) % K + K) % K : j;
      const int jr = right ? j : (j + m + k) % K;
      double tl[4][N], trr[4][N];
      load_canon<N, 4>(M, tr, jl, tl);
      load_canon<N, 4>(M, tr, K + jr, trr);
      double l4[4], r4[4], f4v[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double sl = 0.0, sr = 0.0;
#pragma unroll
        for (int bb = 0; bb < N; ++bb) {
          sl += S.Pf[k][a][bb] * tl[v][bb];
          sr += S.Pf[2 + k][a][bb] * trr[v][bb];
        }
        l4[v] = sl;
        r4[v] = sr;
      }
      const double phi = M.phi0L + S.thL + M.dphi * (jl + S.o[k] + S.s[k] * T.X[a]);
      double sn, cs;
      sincos(phi, &sn, &cs);
      rusanov_d(l4, r4, cs * sc, sn * sc, double(M.gamma), f4v);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        FM[fl][k][a][v] = f4v[v];
        if (VISC) QM[fl][k][a][v] = 0.5 * (l4[v] + r4[v]);
      }
    }
  }
  __syncthreads();
  if (!act) return;
  double acc[4], accq[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) acc[v] = accq[v] = 0.0;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int pb = (right ? 2 : 0) + k;
#pragma unroll
    for (int bb = 0; bb < N; ++bb) {
      const double w = S.Pb[pb][a][bb];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        acc[v] += w * FM[fl][k][bb][v];
        if (VISC) accq[v] += w * QM[fl][k][bb][v];
      }
    }
  }
  const int pa = M.ring_flip[t] ? N - 1 - a : a;
  const double sign = right ? -1.0 : 1.0;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    mflux[(long(t) * N + pa) * 4 + v] = float(sign * acc[v]);
    if (VISC) mqc[(long(t) * N + pa) * 4 + v] = float(accq[v]);
  }
}

template <int N, bool VISC>
__global__ __launch_bounds__(MORTAR_BLOCK) void k_mortar(DevMesh M, OpTables T, MortarTables MT,
                                                         double theta, MortarState *ms_out,
                                                         const float *__restrict__ tr,
                                                         float *__restrict__ mflux,
                                                         float *__restrict__ mqc) {
  mortar_chunk<N, VISC>(M, T, MT, theta, ms_out, tr, mflux, mqc, blockIdx.x);
}

// Canonical point a of ring slot `slot`: C values from a [face][E][point][C]
// trace array, or 4 values from a per-slot record array [slot][point][4].
template <int N, int C>
__device__ __forceinline__ void load_canon_point(const DevMesh &M, const float *__restrict__ tr,
                                                 int slot, int a, double q[C]) {
  const long E = M.E;
  const int e = M.ring_e[slot], f = M.ring_f[slot];
  const int pa = M.ring_flip[slot] ? N - 1 - a : a;
#pragma unroll
  for (int v = 0; v < C; ++v) q[v] = double(tr[((long(f) * E + e) * N + pa) * C + v]);
}

template <int N>
__device__ __forceinline__ void load_slot_point(const DevMesh &M, const float *__restrict__ rec,
                                                int slot, int a, double q[4]) {
  const int pa = M.ring_flip[slot] ? N - 1 - a : a;
#pragma unroll
  for (int v = 0; v < 4; ++v) q[v] = double(rec[(long(slot) * N + pa) * 4 + v]);
}

// Viscous mortar (Sec. 3.2), N lanes per interface face as in k_mortar: each
// side's face viscous flux along the radial (L -> R) normal per unit face
// parameter, from the face's common solution (mqc) and its own gradient
// trace, is projected onto the mortars; the two sides are averaged and the
// mean is projected back to the lane's face point.  Output: outward viscous
// flux, mvflux[slot][point][var].
template <int N>
__device__ __forceinline__ void mortar_visc_chunk(const DevMesh &M, const OpTables &T,
                                                  const MortarState *__restrict__ ms,
                                                  const float *__restrict__ mqc,
                                                  const float *__restrict__ gtr,
                                                  float *__restrict__ mvflux, int chunk) {
  constexpr int FPB = MORTAR_BLOCK / N;
  __shared__ double VF[FPB][2][2][N][4];   // [mortar][side][face point][var]
  __shared__ double VM[FPB][2][N][4];      // averaged flux at the mortar points
  const int K = M.K;
  const int fl = threadIdx.x / N, a = threadIdx.x % N;
  const int t = chunk * FPB + fl;
  const bool act = fl < FPB && t < 2 * K;
  const bool right = t >= K;
  const int j = right ? t - K : t;
  const int m = ms->m;
  const double sc = M.Rs * M.dphi;
  const double mu = M.mu, kT = mu * double(M.gamma) / double(M.prandtl);
  if (act) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int jl = right ? ((j - m - k) % K + K) % K : j;
      const int jr = right ? j : (j + m + k) % K;
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        const int slot = side ? K + jr : jl;
        const int jj = side ? jr : jl;
        const double phi = (side ? M.phi0R + ms->thR : M.phi0L + ms->thL) + M.dphi * (jj + T.X[a]);
        double sn, cs;
        sincos(phi, &sn, &cs);
        double q4[4], g8[8], f[4];
        load_slot_point<N>(M, mqc, slot, a, q4);
        load_canon_point<N, 8>(M, gtr, slot, a, g8);
        visc_flux_n<double>(q4, g8, g8 + 4, cs * sc, sn * sc, mu, kT, f);
#pragma unroll
        for (int v = 0; v < 4; ++v) VF[fl][k][side][a][v] = f[v];
      }
    }
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double sl = 0.0, sr = 0.0;
#pragma unroll
        for (int bb = 0; bb < N; ++bb) {
          sl += ms->Pf[k][a][bb] * VF[fl][k][0][bb][v];
          sr += ms->Pf[2 + k][a][bb] * VF[fl][k][1][bb][v];
        }
        VM[fl][k][a][v] = 0.5 * (sl + sr);
      }
    }
  }
  __syncthreads();
  if (!act) return;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int pb = (right ? 2 : 0) + k;
#pragma unroll
    for (int bb = 0; bb < N; ++bb) {
      const double w = ms->Pb[pb][a][bb];
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[v] += w * VM[fl][k][bb][v];
    }
  }
  const int pa = M.ring_flip[t] ? N - 1 - a : a;
  const double sign = right ? -1.0 : 1.0;
#pragma unroll
  for (int v = 0; v < 4; ++v) mvflux[(long(t) * N + pa) * 4 + v] = float(sign * acc[v]);
}

template <int N>
__global__ __launch_bounds__(MORTAR_BLOCK) void k_mortar_visc(DevMesh M, OpTables T,
                                                              const MortarState *__restrict__ ms,
                                                              const float *__restrict__ mqc,
                                                              const float *__restrict__ gtr,
                                                              float *__restrict__ mvflux) {
  mortar_visc_chunk<N>(M, T, ms, mqc, gtr, mvflux, blockIdx.x);
}

// ---------------------------------------------------------------------------
// dispatch of a runtime N to the kernel templates (N = 2..6)
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

// The same for the orders that also have two-tile blocks (N <= 4).
#define SSD_DISPATCH_N_SMALL(N, CALL)                    \
  switch (N) {                                           \
    case 2: { constexpr int NN = 2; CALL; } break;       \
    case 3: { constexpr int NN = 3; CALL; } break;       \
    case 4: { constexpr int NN = 4; CALL; } break;       \
    default: return hipErrorInvalidValue;                \
  }

}  // namespace ssd

// Internal data structures shared by the host side and the kernels of the
// SSD library.  Nothing here is part of the public ABI (include/ssd.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ssd.h"

namespace ssd {

constexpr int NMAX = 6;

// Packed per-face word, one per (local face, element):
//   bits  0..24  neighbour element (INTERIOR/PERIODIC) or interface slot (SLIDING)
//   bit  25      the neighbour lies in the same block of EB consecutive elements
//   bits 26..27  neighbour's local face
//   bit  28      the neighbour's face parameter runs opposite to ours
//   bits 29..31  SSD_FACE_* kind
constexpr int EB = 64;   // elements per stage-kernel block
__host__ __device__ inline uint32_t pack_face(int kind, int idx, int nf, int rev, int inblock) {
  return (uint32_t(kind) << 29) | (uint32_t(rev & 1) << 28) | (uint32_t(nf & 3) << 26) |
         (uint32_t(inblock & 1) << 25) | (uint32_t(idx) & 0x1FFFFFFu);
}
__host__ __device__ inline int face_kind_of(uint32_t w) { return int(w >> 29); }
__host__ __device__ inline int face_idx_of(uint32_t w) { return int(w & 0x1FFFFFFu); }
__host__ __device__ inline int face_inblock_of(uint32_t w) { return int((w >> 25) & 1u); }
__host__ __device__ inline int face_nf_of(uint32_t w) { return int((w >> 26) & 3u); }
__host__ __device__ inline int face_rev_of(uint32_t w) { return int((w >> 28) & 1u); }
// A face's trace is read by another block (or by the mortar kernel) and must
// be stored: sliding faces, and conforming faces whose neighbour is elsewhere.
__host__ __device__ inline bool face_exported(uint32_t w) {
  const int k = face_kind_of(w);
  return k == SSD_FACE_SLIDING ||
         ((k == SSD_FACE_INTERIOR || k == SSD_FACE_PERIODIC) && !face_inblock_of(w));
}
constexpr int MAX_ELEMS = 1 << 25;
constexpr int TRACE_BLOCK = 256;   // elements per block of the trace kernel

// Element flag word: bit 0 cubic map, bit 1 rotating zone, bits 8.. cubic slot.
constexpr int EF_CUBIC = 1;
constexpr int EF_ROT = 2;

// 1-D operator tables in FP32 for the kernels (interpolation and
// derivative of eqs. Qt, Ft, Gt), the point sets in FP64 for the metrics.
struct OpTables {
  float I[NMAX + 1][NMAX];   // I[k][i] = h_i(Xf_k)
  float D[NMAX][NMAX + 1];   // D[i][k] = l'_k(X_i)
  double X[NMAX];            // solution points
  double Xf[NMAX + 1];       // flux points
};

// Tables for the device-side mortar rebuild (FP64).
struct MortarTables {
  double X[NMAX];            // solution points (mortar and face share them)
  double bw[NMAX];           // barycentric weights of X
  double zq[NMAX];           // N-point Gauss-Legendre nodes on [0,1]
  double wq[NMAX];           // and weights
  double hq[NMAX][NMAX];     // hq[q][i] = h_i(zq[q])
  double Minv[NMAX][NMAX];   // inverse mortar mass matrix (eq. mortarM)
};

// Mortar placement and projections for the current angle, written by the
// rebuild kernel.  Index k: 0 L-side mortar 1, 1 L-side mortar 2,
// 2 R-side mortar 1, 3 R-side mortar 2.
struct MortarState {
  int m;
  int valid;
  double delta;
  double thL, thR;
  double o[4], s[4];
  double Pf[4][NMAX][NMAX];   // M^-1 A(o,s)          (eq. prjQ2)
  double Pb[4][NMAX][NMAX];   // s M^-1 A(o,s)^T      (eq. prjF2)
};

// Everything the kernels need about one mesh (passed by value).
struct DevMesh {
  int E;           // elements
  int K;           // faces per interface side (0: no interface)
  int C;           // cubic elements
  int N;
  const float *geo;        // [8][E]: bilinear map p0, A, C, T (x, y each), see load_geo
  const int *eflag;        // [E]
  const uint32_t *face;    // [4][E]
  const double *cmet;      // cubic-cell metrics, see cubic_index()
  const int *ring_e;       // [2K] L slots 0..K-1, R slots K..2K-1 (CCW order)
  const int *ring_f;       // [2K]
  const int *ring_flip;    // [2K]
  int *flag;               // numeric-failure flag
  float gamma, gas_R, mu, prandtl, T_wall;
  float qinf[4];
  double phi0L, phi0R, dphi, Rs;
  int rotL, rotR;
};

// Layout of the cubic-cell metric array (FP64, body frame, positions
// relative to the rotation centre), cubic slot fastest:
//   xi-FPs  (j, k), quantities 0 x_eta, 1 y_eta, 2 x, 3 y
//   eta-FPs (k, i), quantities 0 x_xi, 1 y_xi, 2 x, 3 y
//   SPs     (j, i), quantities 0 |J|, 1 x_xi, 2 x_eta, 3 y_xi, 4 y_eta
__host__ __device__ inline long cubic_xi_index(int N, int C, int q, int j, int k, int c) {
  return ((long(q) * N + j) * (N + 1) + k) * C + c;
}
__host__ __device__ inline long cubic_eta_index(int N, int C, int q, int k, int i, int c) {
  return 4L * N * (N + 1) * C + ((long(q) * (N + 1) + k) * N + i) * C + c;
}
__host__ __device__ inline long cubic_sp_index(int N, int C, int q, int j, int i, int c) {
  return 8L * N * (N + 1) * C + ((long(q) * N + j) * N + i) * C + c;
}
__host__ __device__ inline long cubic_len(int N, int C) {
  return (8L * N * (N + 1) + 5L * N * N) * C;
}

// Per-call rotation of zone 1 (cos, sin of theta, and omega).
struct Rotation {
  double ct, st, omega;
};

// Face data buffer of a state (two per handle, one per RK stage parity), in
// floats: the exported face traces [face][E][point][4] (16 N E), the mortar
// flux of the interface faces [slot][point][4] (8 K N), and on viscous
// meshes the mortar common solution [slot][point][4] (8 K N).
inline long face_trace_floats(int N, int E) { return 16L * N * E; }
inline long face_record_floats(int N, int K) { return 8L * K * N; }
inline long face_buffer_floats(int N, int E, int K) {
  return face_trace_floats(N, E) + 2 * face_record_floats(N, K);
}

// Viscous work buffers (device, owned by the mesh handle).
struct ViscIO {
  float *G;        // grad Q at the SPs [(c*4+v)][j][i][E], c = 0 x, 1 y
  float *gtr;      // gradient traces [face][E][point][8]
  float *mvflux;   // viscous mortar flux [slot][point][4]
};

// Kernel launchers (single mesh: ssd_kernels.hip; batched: ssd_batch.hip).
hipError_t launch_traces(const DevMesh &M, const OpTables &T, const float *q, float *tr,
                         hipStream_t s);
hipError_t launch_rebuild(const DevMesh &M, const MortarTables &MT, double theta, MortarState *ms,
                          hipStream_t s);
// Rebuilds the mortars for theta (stored to ms) and forms the inviscid
// mortar flux; mqc may be null (inviscid), else it also receives the
// mortar common solution.
hipError_t launch_mortar(const DevMesh &M, const OpTables &T, const MortarTables &MT,
                         double theta, MortarState *ms, const float *tr, float *mflux, float *mqc,
                         hipStream_t s);
// facein: face data buffer of q with its traces and mortar common solution.
hipError_t launch_grad(const DevMesh &M, const OpTables &T, Rotation rot, const float *q,
                       const float *facein, float *G, float *gtr, hipStream_t s);
hipError_t launch_mortar_visc(const DevMesh &M, const OpTables &T, const MortarState *ms,
                              const float *mqc, const float *gtr, float *mvflux, hipStream_t s);
// Coefficients of one Runge-Kutta stage: out = qn + beta (q - qn) +
// gamma dt dQ/dt [+ add] (qn null: qn = q).
struct RKCoef {
  float beta, gamma, dt;
  const float *add;   // null: nothing added
};

// facein: face data buffer of q with its traces and mortar flux; trout:
// the face data buffer the new state's traces go to (rk).  visc null:
// inviscid residual.
hipError_t launch_stage(const DevMesh &M, const OpTables &T, Rotation rot, const float *q,
                        const float *qn, float *out, const float *facein, float *trout,
                        const ViscIO *visc, const RKCoef &C, bool rk, hipStream_t s);
// ---------------------------------------------------------------------------
// batched execution of many meshes (same device): per-case descriptors and
// work tables live in device memory; every batched kernel walks a table of
// (case, tile or chunk) pairs with a grid-stride loop.
// ---------------------------------------------------------------------------
struct BatchCase {
  DevMesh M;
  double theta0, omega;   // rotor motion: theta = theta0 + omega t
  double t0, dt;          // step n starts at t0 + n dt
  MortarState *ms;
  float *buf[4];          // stage arrays: 0 the state, 1..3 the work arrays
  float *face[2];         // face data buffers
  ViscIO V;
};

// Which stage arrays a batched stage reads and writes (indices into
// BatchCase::buf, -1: none), the face buffer parity and the stage time
// offset c (theta at t0 + (n + c) dt, n read from the step counter).
struct BatchStage {
  int in, qn, out, add;
  int cur;
  float beta, gamma;
  double c;
};

// Batched launchers: one block per item of `work`, a table of (case, tile
// or chunk) pairs; `step` points at the group's step counter.
hipError_t launch_batch_traces(int N, const BatchCase *cases, const uint2 *work, int nwork,
                               const OpTables &T, hipStream_t s);
hipError_t launch_batch_mortar(int N, bool visc, const BatchCase *cases, const uint2 *work,
                               int nwork, const OpTables &T, const MortarTables &MT, int cur,
                               double c, const double *step, hipStream_t s);
hipError_t launch_batch_grad(int N, const BatchCase *cases, const uint2 *work, int nwork,
                             const OpTables &T, int in, int cur, double c, const double *step,
                             hipStream_t s);
hipError_t launch_batch_mortar_visc(int N, const BatchCase *cases, const uint2 *work, int nwork,
                                    const OpTables &T, int cur, hipStream_t s);
hipError_t launch_batch_stage(int N, bool visc, const BatchCase *cases, const uint2 *work,
                              int nwork, const OpTables &T, const BatchStage &S,
                              const double *step, hipStream_t s);
hipError_t launch_batch_combine(const BatchCase *cases, const uint2 *work, int nwork, float w2,
                                float w3, float w4, hipStream_t s);
hipError_t launch_step_count(double *step, hipStream_t s);

// ---------------------------------------------------------------------------
// learned per-element subgrid correction (ssd_mlp.hip)
// ---------------------------------------------------------------------------
constexpr int MLP_HIDDEN = SSD_MLP_HIDDEN;

// Read-only view of a network for the kernels.  bf16 weights, row-major with
// padded widths KIN = 32 ceil(n_in / 32), KOUT = 32 ceil(n_out / 32):
// W1 [H][KIN], W2 [H][H], W3 [KOUT][H], and the transposed W2t [H][H]
// (W2t[i][o] = W2[o][i]) and W3t [H][KOUT].  FP32 biases and the
// normalisation (padding entries 0, isig 0).
struct MlpDev {
  const __bf16 *W1, *W2, *W3, *W2t, *W3t;
  const float *b1, *b2, *b3;
  const float *mu_x, *isig_x;   // [KIN]
  const float *mu_y, *sig_y;    // [KOUT]
};

// Gradient accumulators (FP32, same padded shapes) and the loss sum.
struct MlpGrad {
  float *W1, *W2, *W3, *b1, *b2, *b3;
  double *loss;
};

// Flat FP32 parameters [W1 | b1 | W2 | b2 | W3 | b3] with their gradient and
// Adam moments, and where the bf16 copies go.
struct MlpStore {
  float *P, *G, *M, *V;
  __bf16 *W1b, *W2b, *W3b, *W2tb, *W3tb;
  long o_b1, o_W2, o_b2, o_W3, o_b3;
  int kin, kout;
};

// 1-D restriction operators r[a][ic][if] of the two child halves.
struct Restrict1D {
  float r[2][NMAX][NMAX];
};

hipError_t launch_features(const DevMesh &M, const OpTables &T, const float *q, float *X,
                           hipStream_t s);
// add[o][e] = scale * (MLP correction of element e), o in the state layout
hipError_t launch_subgrid(const DevMesh &M, const OpTables &T, const MlpDev &P, const float *q,
                          float *add, float scale, hipStream_t s);
hipError_t launch_mlp_forward(int N, const MlpDev &P, const float *X, long n, float *Y,
                              hipStream_t s);
// adds the minibatch's loss gradient to G and its mean loss to *G.loss;
// rows idx[s] outside [0, n_rows) are skipped
hipError_t launch_mlp_grad(int N, const MlpDev &P, const MlpGrad &G, const float *X,
                           const float *Tg, long n_rows, const int *idx, int batch,
                           hipStream_t s);
hipError_t launch_adam(const MlpStore &S, long n, float lr, float b1, float b2, float eps,
                       float bc1, float bc2, hipStream_t s);
hipError_t launch_mlp_sync(const MlpStore &S, long n, hipStream_t s);
hipError_t launch_moments(const float *A, long n, int cols, double *acc, hipStream_t s);
// out = restriction of qf (nested fine state) - sub (null: nothing); rows:
// out[c][o], else the state layout out[o][c]
hipError_t launch_restrict(int Nc, int Nf, const float *qf, long Ef, const int *children, long Ec,
                           const Restrict1D &R, const float *sub, float *out, bool rows,
                           hipStream_t s);

// W = w2 (u2 - un) + w3 (u3 - un) + w4 (u4 - un) over n floats.
hipError_t launch_rk_combine(long n, const float *un, const float *u2, const float *u3,
                             const float *u4, float w2, float w3, float w4, float *W,
                             hipStream_t s);

}  // namespace ssd

// Launchers of the SSD kernels and the host-side descriptors of batched and
// learned-correction work (single mesh: ssd_kernels.hip; batched:
// ssd_batch.hip; learned correction: ssd_mlp.hip).  Nothing here is part
// of the public ABI.
#pragma once

#include "ssd_internal.h"

namespace ssd {

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
// reverse: tiles taken in reverse block order.
hipError_t launch_grad(const DevMesh &M, const OpTables &T, Rotation rot, const float *q,
                       const float *facein, float *G, float *gtr, hipStream_t s,
                       bool reverse = false);
hipError_t launch_mortar_visc(const DevMesh &M, const OpTables &T, const MortarState *ms,
                              const float *mqc, const float *gtr, float *mvflux, hipStream_t s);
// facein: face data buffer of q with its traces and mortar flux; trout:
// the face data buffer the new state's traces go to (rk).  visc null:
// inviscid residual.
hipError_t launch_stage(const DevMesh &M, const OpTables &T, Rotation rot, const float *q,
                        const float *qn, float *out, const float *facein, float *trout,
                        const ViscIO *visc, const RKCoef &C, bool rk, hipStream_t s,
                        hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
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
  // SSPRK54's fourth stage: the stage array that holds U2 and receives the
  // last stage's increment W = cw2 (U2 - Qn) + cw3 (Q - Qn) + cw4 (Q_new - Qn)
  int comb = -1;
  float cw2 = 0.0f, cw3 = 0.0f, cw4 = 0.0f;
  // nonzero: the work table is taken in reverse order (successive stages of
  // a viscous group alternate, so a stage starts on the tiles the previous
  // one touched last; inviscid groups run forward)
  int reverse = 0;
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
// tpb: work items (64-cell tiles) per block, 1, or 2 for N <= 4
hipError_t launch_batch_stage(int N, bool visc, const BatchCase *cases, const uint2 *work,
                              int nwork, const OpTables &T, const BatchStage &S,
                              const double *step, hipStream_t s, int tpb = 1);
hipError_t launch_step_count(double *step, hipStream_t s);

// the contraction probe (ssd_probe.hip): N = 4 operators of T
hipError_t launch_probe(int variant, const OpTables &T, int n_cells, int reps, const float *q,
                        float *out, hipStream_t s);
// the stream probe (ssd_probe.hip): c = 0.75 a + 0.25 b over n floats
hipError_t launch_stream_probe(int variant, int64_t n, const float *a, const float *b, float *c,
                               hipStream_t s);

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
// rows idx[s] outside [0, n_rows) are skipped; noise: standard deviation of
// the uniform input noise of stream seed at training step `step`
hipError_t launch_mlp_grad(int N, const MlpDev &P, const MlpGrad &G, const float *X,
                           const float *Tg, long n_rows, const int *idx, int batch, float noise,
                           uint64_t seed, uint64_t step, hipStream_t s);
hipError_t launch_adam(const MlpStore &S, long n, float lr, float b1, float b2, float eps,
                       float bc1, float bc2, hipStream_t s);
hipError_t launch_mlp_sync(const MlpStore &S, long n, hipStream_t s);
hipError_t launch_moments(const float *A, long n, int cols, double *acc, hipStream_t s);
// rows T[e][o] += rate (qa - qb), qa and qb in the cell-blocked state layout
hipError_t launch_nudge(const float *qa, const float *qb, long E, int planes, float rate, float *T,
                        hipStream_t s);
// out = restriction of qf (nested fine state; children null: the same mesh
// at a lower order) - sub (null: nothing); rows: out[c][o], else the state
// layout out[o][c]
hipError_t launch_restrict(int Nc, int Nf, const float *qf, long Ef, const int *children, long Ec,
                           const Restrict1D &R, const float *sub, float *out, bool rows,
                           hipStream_t s);

// ---------------------------------------------------------------------------
// general sliding interface (ssd_iface.hip): sides of KL and KR faces, any
// widths.  L faces use ring slots 0..KL-1, R faces K..K+KR-1 (DevMesh::K =
// max(KL, KR)).
// ---------------------------------------------------------------------------
struct GenRing {
  int KL, KR;
  const double *start;   // [KL] then [KR]: canonical (counter-clockwise) face start
                         // angles in the body frame, ascending in [0, 2 pi)
  const double *width;   // [KL] then [KR]: the faces' angular widths
  double *mb;            // [KL + KR] merged rotated starts (the mortar start angles)
  int *msrc;             // [KL + KR] side << 30 | sorted-rotated index of each
  int *posL, *posR;      // [KL], [KR] merged position of each sorted-rotated start
  double *mf;            // [KL + KR][N][4] mortar flux per unit angle times R
  double *mq;            // [KL + KR][N][4] mortar common solution (viscous meshes)
};

// Rotor angle of a general-ring launch: `theta`, or, with `bc` set, the
// batched case's angle at stage offset c of step *step (read on the device,
// so that a captured graph follows the step counter).
struct AngleArg {
  double theta;
  const BatchCase *bc;
  double c;
  const double *step;
};
__device__ __forceinline__ double angle_value(const AngleArg &A) {
  if (!A.bc) return A.theta;
  const BatchCase &B = *A.bc;
  return B.theta0 + B.omega * (B.t0 + (A.step[0] + A.c) * B.dt);
}

// Mortar merge, mortar fluxes and their projection back to the faces for
// the rotor angle A (tr: the face data buffer's traces); with mqc also the
// faces' common solution.
hipError_t launch_gen_mortar(const DevMesh &M, const OpTables &T, const MortarTables &MT,
                             const GenRing &G, const AngleArg &A, const float *tr, float *mflux,
                             float *mqc, hipStream_t s);
// Viscous mortar flux from the faces' common solution and gradient traces,
// for the angle of the preceding launch_gen_mortar.
hipError_t launch_gen_mortar_visc(const DevMesh &M, const OpTables &T, const MortarTables &MT,
                                  const GenRing &G, const AngleArg &A, const float *mqc,
                                  const float *gtr, float *mvflux, hipStream_t s);

}  // namespace ssd

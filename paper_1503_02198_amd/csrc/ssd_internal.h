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
constexpr int MORTAR_BLOCK = 64;   // threads per mortar workgroup, N per interface face

// Cell-blocked layout of per-cell arrays of `planes` values each (a state:
// planes = 4 N^2, plane (v N + j) N + i holds Q[v] at solution point
// (X_i, X_j)).  Cells go in blocks of EB consecutive cells, the last block
// holding the remaining E mod EB; block b stores its values plane after
// plane, each plane as one row of its nb = min(EB, E - EB b) cells.  A
// stage-kernel block therefore reads and writes one contiguous span.
__host__ __device__ inline long cb_rows(long b, long E) {
  return E - long(EB) * b < EB ? E - long(EB) * b : EB;
}
__host__ __device__ inline long cb_index(long e, long p, long planes, long E) {
  const long b = e / EB;
  return b * EB * planes + p * cb_rows(b, E) + (e - b * EB);
}
// the same in 32-bit arithmetic, for arrays of fewer than 2^32 values (the
// per-cell geometry and face words, which use the same blocking)
__host__ __device__ inline uint32_t cb_index32(uint32_t e, uint32_t p, uint32_t planes, uint32_t E) {
  const uint32_t b = e / EB, r = E - EB * b;
  return b * EB * planes + p * (r < uint32_t(EB) ? r : uint32_t(EB)) + (e - b * EB);
}
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
// be stored: sliding faces, and conforming faces without the in-block bit
// (set where the neighbour is in the same 64-element block, across a face of
// the same direction with the same point order).
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
  const float *geo;        // 8 planes, cell-blocked: bilinear map p0, A, C, T (x, y each), see load_geo
  const int *eflag;        // [E]
  const uint32_t *face;    // 4 planes (local faces), cell-blocked
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

// Coefficients of one Runge-Kutta stage: out = qn + beta (q - qn) +
// gamma dt dQ/dt [+ add_scale add] (qn null: qn = q).
struct RKCoef {
  float beta, gamma, dt;
  const float *add;        // null: nothing added
  float add_scale = 1.0f;
  // nonzero: tiles taken in reverse block order, so that a launch starts on
  // the cells the previous launch touched last (still in the memory-side
  // cache), except that tiles 0 .. lead - 1 come first, in order
  int reverse = 0;
  int lead = 0;
  // SSPRK54, fourth stage: with comb set, the stage also forms the last
  // stage's increment W = cw2 (U2 - Qn) + cw3 (Q - Qn) + cw4 (Q_new - Qn),
  // reading U2 from comb and writing W over it
  float *comb = nullptr;
  float cw2 = 0.0f, cw3 = 0.0f, cw4 = 0.0f;
};

}  // namespace ssd

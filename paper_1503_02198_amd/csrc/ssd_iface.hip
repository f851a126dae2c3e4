// General sliding interface on gfx950: rings whose sides have different face
// counts and non-uniform faces, so that a face meets any number of mortars
// (the extension named at the end of Sec. 3.2 and in the conclusions).
//
// Per stage, for the rotor angle:
//   1. k_gen_merge: the two sides' face start angles, rotated and sorted
//      (each side's order is a cyclic shift of its stored order), are merged
//      by rank: every start finds its merged position by binary search in
//      the other side (ties: the L start first).  Consecutive merged starts
//      bound the M = KL + KR mortars; each lies on one L and one R face.
//   2. k_gen_flux: per mortar point, both sides' traces are projected onto
//      the mortar (M^-1 A(o, s), eq. prjQ2, with the mortar's own offset o
//      and length s on each face, in FP64) and the Rusanov flux is taken on
//      the exact circle, per unit angle times R.
//   3. k_gen_back: per face point, the face's mortars (consecutive in the
//      merged order) are projected back (s M^-1 A^T, eq. prjF2) and scaled
//      by the face's angular width, giving the outward flux per unit face
//      parameter in the records the stage kernel reads.
// Viscous meshes: k_gen_flux also keeps the mean of the two projections
// (BR1 common solution), projected back into the common-solution records;
// after the gradient pass k_gen_vflux averages the two sides' face viscous
// fluxes on each mortar, and k_gen_back projects them back.
#include "ssd_launch.h"
#include "ssd_tiles.h"

namespace ssd {

constexpr double TWO_PI = 6.283185307179586476925;

__device__ __forceinline__ double wrap_2pi(double a) {
  a = fmod(a, TWO_PI);
  return a < 0.0 ? a + TWO_PI : a;
}

// Sorted-rotated access to one side: the faces' rotated start angles in
// ascending order are start[(t + r) mod K] + th (wrapped), t = 0..K-1.
struct SideView {
  const double *start, *width;
  int K, r;
  double th;
  __device__ double angle(int t) const { return wrap_2pi(start[(t + r) % K] + th); }
  __device__ int face(int t) const { return (t + r) % K; }
};

// First stored index whose rotated start wraps past 2 pi (0 if none):
// where the ascending order of the rotated starts begins.
__device__ __forceinline__ int rotation_of(const double *start, int K, double th) {
  const double t = wrap_2pi(th);
  int lo = 0, hi = K;   // first i with start[i] + t >= 2 pi
  while (lo < hi) {
    const int mid = (lo + hi) / 2;
    if (start[mid] + t >= TWO_PI) hi = mid; else lo = mid + 1;
  }
  return lo == K ? 0 : lo;
}

__device__ __forceinline__ SideView side_view(const GenRing &G, int side, double theta,
                                              const DevMesh &M) {
  SideView v;
  v.start = G.start + (side ? G.KL : 0);
  v.width = G.width + (side ? G.KL : 0);
  v.K = side ? G.KR : G.KL;
  v.th = (side ? M.rotR : M.rotL) ? theta : 0.0;
  v.r = rotation_of(v.start, v.K, v.th);
  return v;
}

// number of entries of `o` below x (strict) or at most x
__device__ __forceinline__ int rank_in(const SideView &o, double x, bool strict) {
  int lo = 0, hi = o.K;
  while (lo < hi) {
    const int mid = (lo + hi) / 2;
    const double a = o.angle(mid);
    if (strict ? a < x : a <= x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(256) void k_gen_merge(DevMesh M, GenRing G, AngleArg A) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= G.KL + G.KR) return;
  const double theta = angle_value(A);
  const int side = i < G.KL ? 0 : 1;
  const int t = side ? i - G.KL : i;
  const SideView own = side_view(G, side, theta, M), other = side_view(G, side ^ 1, theta, M);
  const double a = own.angle(t);
  const int pos = t + rank_in(other, a, side == 0);
  G.mb[pos] = a;
  G.msrc[pos] = (side << 30) | t;
  (side ? G.posR : G.posL)[t] = pos;
}

// A(i, j) = int_0^1 h_i(z) h_j(o + s z) dz (i mortar basis, j face basis)
template <int N>
__device__ __forceinline__ void overlap(const MortarTables &MT, double o, double s,
                                        double (&A)[N][N]) {
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) A[i][j] = 0.0;
  for (int q = 0; q < N; ++q) {
    const double x = o + s * MT.zq[q];
    double hj[N];
#pragma unroll
    for (int j = 0; j < N; ++j) hj[j] = lagrange_d(MT, N, j, x);
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = 0; j < N; ++j) A[i][j] += MT.wq[q] * MT.hq[q][i] * hj[j];
  }
}

// The mortar at merged position k: its L and R faces (stored indices) and
// its offset and length on each, its start angle and width.
struct MortarRec {
  int f[2];
  double o[2], s[2];
  double b0, w;
};

__device__ __forceinline__ MortarRec mortar_at(const DevMesh &M, const GenRing &G, double theta,
                                               int k) {
  const int Mn = G.KL + G.KR;
  const SideView v[2] = {side_view(G, 0, theta, M), side_view(G, 1, theta, M)};
  MortarRec r;
  r.b0 = G.mb[k];
  const double b1 = k + 1 < Mn ? G.mb[k + 1] : G.mb[0] + TWO_PI;
  r.w = fmax(b1 - r.b0, 0.0);
  const int src = G.msrc[k];
  const int sd = src >> 30, t = src & 0x3FFFFFFF;
  int n[2];   // starts of each side at merged positions <= k
  n[sd] = t + 1;
  n[sd ^ 1] = k - t;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int ts = n[s] > 0 ? n[s] - 1 : v[s].K - 1;   // before the first start: the last face
    const int face = v[s].face(ts);
    const double width = v[s].width[face];
    r.f[s] = face;
    r.o[s] = wrap_2pi(r.b0 - v[s].angle(ts)) / width;
    r.s[s] = r.w / width;
  }
  return r;
}

template <int N, bool VISC>
__global__ __launch_bounds__(256) void k_gen_flux(DevMesh M, OpTables T, MortarTables MT,
                                                  GenRing G, AngleArg Ang,
                                                  const float *__restrict__ tr) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  const int Mn = G.KL + G.KR;
  if (idx >= Mn * N) return;
  const double theta = angle_value(Ang);
  const int k = idx / N, a = idx % N;
  const MortarRec r = mortar_at(M, G, theta, k);
  double q[2][4];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    double A[N][N];
    overlap<N>(MT, r.o[s], r.s[s], A);
    double tf[4][N];
    load_canon<N, 4>(M, tr, s ? M.K + r.f[s] : r.f[s], tf);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      double acc = 0.0;
#pragma unroll
      for (int b = 0; b < N; ++b) {
        double pf = 0.0;   // (M^-1 A)[a][b]
#pragma unroll
        for (int l = 0; l < N; ++l) pf += MT.Minv[a][l] * A[l][b];
        acc += pf * tf[v][b];
      }
      q[s][v] = acc;
    }
  }
  double sn, cs;
  sincos(r.b0 + r.w * T.X[a], &sn, &cs);
  double f4[4];
  rusanov_d(q[0], q[1], cs * M.Rs, sn * M.Rs, double(M.gamma), f4);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    G.mf[(long(k) * N + a) * 4 + v] = f4[v];
    // BR1 common solution at the mortar point: the mean of both projections
    if (VISC) G.mq[(long(k) * N + a) * 4 + v] = 0.5 * (q[0][v] + q[1][v]);
  }
}

// Viscous mortar flux at mortar point a: each side's face viscous flux along
// the radial normal per unit angle times R, at its face points from the
// face's common solution (mqc) and own gradient trace (gtr), projected onto
// the mortar; the two sides averaged.  Into G.mf.
template <int N>
__global__ __launch_bounds__(256) void k_gen_vflux(DevMesh M, OpTables T, MortarTables MT,
                                                   GenRing G, AngleArg Ang,
                                                   const float *__restrict__ mqc,
                                                   const float *__restrict__ gtr) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  const int Mn = G.KL + G.KR;
  if (idx >= Mn * N) return;
  const double theta = angle_value(Ang);
  const int k = idx / N, a = idx % N;
  const MortarRec r = mortar_at(M, G, theta, k);
  const double mu = M.mu, kT = mu * double(M.gamma) / double(M.prandtl);
  double avg[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int slot = s ? M.K + r.f[s] : r.f[s];
    const double *start = G.start + (s ? G.KL : 0), *width = G.width + (s ? G.KL : 0);
    const double th = (s ? M.rotR : M.rotL) ? theta : 0.0;
    double vf[4][N];
#pragma unroll
    for (int b = 0; b < N; ++b) {
      double sn, cs;
      sincos(start[r.f[s]] + th + width[r.f[s]] * T.X[b], &sn, &cs);
      double q4[4], g8[8], f[4];
      load_slot_point<N>(M, mqc, slot, b, q4);
      load_canon_point<N, 8>(M, gtr, slot, b, g8);
      visc_flux_n<double>(q4, g8, g8 + 4, cs * M.Rs, sn * M.Rs, mu, kT, f);
#pragma unroll
      for (int v = 0; v < 4; ++v) vf[v][b] = f[v];
    }
    double A[N][N];
    overlap<N>(MT, r.o[s], r.s[s], A);
#pragma unroll
    for (int b = 0; b < N; ++b) {
      double pf = 0.0;   // (M^-1 A)[a][b]
#pragma unroll
      for (int l = 0; l < N; ++l) pf += MT.Minv[a][l] * A[l][b];
#pragma unroll
      for (int v = 0; v < 4; ++v) avg[v] += 0.5 * pf * vf[v][b];
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) G.mf[(long(k) * N + a) * 4 + v] = avg[v];
}

// Back-projection of mortar data src [M][N][4] to face records dst: for a
// flux, outward and per unit face parameter (times the face width, R faces
// negated); for the common solution, as it is.
template <int N>
__global__ __launch_bounds__(256) void k_gen_back(DevMesh M, MortarTables MT, GenRing G,
                                                  AngleArg Ang, const double *__restrict__ src,
                                                  float *__restrict__ dst, int flux) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= (G.KL + G.KR) * N) return;
  const double theta = angle_value(Ang);
  const int i = idx / N, a = idx % N;
  const int side = i < G.KL ? 0 : 1;
  const int face = side ? i - G.KL : i;
  const int Mn = G.KL + G.KR;
  const SideView v = side_view(G, side, theta, M);
  const int t = ((face - v.r) % v.K + v.K) % v.K;   // sorted-rotated index of the face
  const int *pos = side ? G.posR : G.posL;
  const int p0 = pos[t], p1 = t + 1 < v.K ? pos[t + 1] : pos[0] + Mn;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int p = p0; p < p1; ++p) {
    const int k = p % Mn;
    const MortarRec r = mortar_at(M, G, theta, k);
    if (!(r.s[side] > 0.0)) continue;
    double A[N][N];
    overlap<N>(MT, r.o[side], r.s[side], A);
#pragma unroll
    for (int b = 0; b < N; ++b) {
      double pb = 0.0;   // (s M^-1 A^T)[a][b]
#pragma unroll
      for (int l = 0; l < N; ++l) pb += MT.Minv[a][l] * A[b][l];
      pb *= r.s[side];
#pragma unroll
      for (int vv = 0; vv < 4; ++vv) acc[vv] += pb * src[(long(k) * N + b) * 4 + vv];
    }
  }
  const int slot = side ? M.K + face : face;
  const int pa = M.ring_flip[slot] ? N - 1 - a : a;
  const double sc = flux ? (side ? -1.0 : 1.0) * v.width[face] : 1.0;
#pragma unroll
  for (int vv = 0; vv < 4; ++vv) dst[(long(slot) * N + pa) * 4 + vv] = float(sc * acc[vv]);
}

hipError_t launch_gen_mortar(const DevMesh &M, const OpTables &T, const MortarTables &MT,
                             const GenRing &G, const AngleArg &A, const float *tr, float *mflux,
                             float *mqc, hipStream_t s) {
  const int nb = G.KL + G.KR;
  hipLaunchKernelGGL(k_gen_merge, dim3((nb + 255) / 256), dim3(256), 0, s, M, G, A);
  const int np = nb * M.N;
  const dim3 grid((np + 255) / 256);
  if (mqc) {
    SSD_DISPATCH_N(M.N, hipLaunchKernelGGL((k_gen_flux<NN, true>), grid, dim3(256), 0, s, M, T,
                                           MT, G, A, tr));
  } else {
    SSD_DISPATCH_N(M.N, hipLaunchKernelGGL((k_gen_flux<NN, false>), grid, dim3(256), 0, s, M, T,
                                           MT, G, A, tr));
  }
  SSD_DISPATCH_N(M.N, hipLaunchKernelGGL(k_gen_back<NN>, grid, dim3(256), 0, s, M, MT, G, A,
                                         G.mf, mflux, 1));
  if (mqc)
    SSD_DISPATCH_N(M.N, hipLaunchKernelGGL(k_gen_back<NN>, grid, dim3(256), 0, s, M, MT, G, A,
                                           G.mq, mqc, 0));
  return hipGetLastError();
}

hipError_t launch_gen_mortar_visc(const DevMesh &M, const OpTables &T, const MortarTables &MT,
                                  const GenRing &G, const AngleArg &A, const float *mqc,
                                  const float *gtr, float *mvflux, hipStream_t s) {
  const int np = (G.KL + G.KR) * M.N;
  const dim3 grid((np + 255) / 256);
  SSD_DISPATCH_N(M.N, hipLaunchKernelGGL(k_gen_vflux<NN>, grid, dim3(256), 0, s, M, T, MT, G,
                                         A, mqc, gtr));
  SSD_DISPATCH_N(M.N, hipLaunchKernelGGL(k_gen_back<NN>, grid, dim3(256), 0, s, M, MT, G, A,
                                         G.mf, mvflux, 1));
  return hipGetLastError();
}

}  // namespace ssd

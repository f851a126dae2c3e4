// Learned per-element subgrid correction on gfx950 (an extension of the
// method, not in the paper): element features, restriction of a nested fine
// mesh to its coarse parent, and a small MLP whose products run on the BF16
// matrix cores with FP32 accumulation.
//
// MLP: xn = (x - mu_x) / sig_x -> h1 = tanh(W1 xn + b1) -> h2 = tanh(W2 h1 +
// b2) -> yn = W3 h2 + b3 -> y = yn sig_y + mu_y, hidden width H = 64.  The
// operands of every product (xn, h1, h2, the weights and, in the backward
// pass, the output and hidden-layer gradients) are rounded to bfloat16; the
// products accumulate in FP32; biases, tanh and the loss stay in FP32.
//
// Matrix products use v_mfma_f32_16x16x32_bf16 over a block of 64 rows
// (samples or elements) and 4 waves; in the forward pass wave w owns rows
// 16w..16w+15.  Operand layout of the 16x16x32 product D = A B:
//   A (16 x 32): lane l holds A[l % 16][8 (l / 16) + e], e = 0..7
//   B (32 x 16): lane l holds B[8 (l / 16) + e][l % 16]
//   D (16 x 16): lane l holds D[4 (l / 16) + r][l % 16], r = 0..3
#include "ssd_device.h"
#include "ssd_launch.h"

namespace ssd {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// bfloat16 from FP32, round to nearest with ties to even (finite inputs)
__device__ __forceinline__ __bf16 to_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  const unsigned short h = static_cast<unsigned short>(u >> 16);
  return __builtin_bit_cast(__bf16, h);
}
__device__ __forceinline__ float from_bf16(__bf16 h) {
  return __uint_as_float(uint32_t(__builtin_bit_cast(unsigned short, h)) << 16);
}

// Training noise: SplitMix64 (Steele, Lea and Flood, 2014) output for
// counter c of stream `seed` (the mix of seed + (c + 1) 0x9E3779B97F4A7C15),
// its top 24 bits as u in [0, 1), and eps = (2u - 1) sqrt(3), uniform with
// unit variance; every step is exact in FP32.
__device__ __forceinline__ float noise_eps(uint64_t seed, uint64_t c) {
  uint64_t z = seed + (c + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  const float u = float(uint32_t(z >> 40)) * 0x1p-24f;
  return (2.0f * u - 1.0f) * 1.7320508075688772f;
}

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Sizes of the network for meshes of N solution points per direction.
template <int N>
struct MlpDims {
  static constexpr int NIN = 4 * N * N + 16 * N;          // features
  static constexpr int NOUT = 4 * N * N;                  // outputs
  static constexpr int KIN = (NIN + 31) / 32 * 32;        // padded to the product depth
  static constexpr int KOUT = (NOUT + 31) / 32 * 32;
  static constexpr int H = MLP_HIDDEN;
};

// ---------------------------------------------------------------------------
// products over a block's 64 rows
// ---------------------------------------------------------------------------
// acc[nt] += A[r0 + 0..15][0..K) * W[16 nt + 0..15][0..K)^T, A in LDS with
// row stride lda, W in global memory with row stride ldw (bf16 elements).
template <int K, int NT>
__device__ __forceinline__ void rows_times_wt(const __bf16 *A, int lda, const __bf16 *W, int ldw,
                                              int r0, f32x4 (&acc)[NT]) {
  const int l = threadIdx.x & 63;
  const int kq = (l >> 4) * 8;
#pragma unroll
  for (int k0 = 0; k0 < K; k0 += 32) {
    const bf16x8 a = *reinterpret_cast<const bf16x8 *>(A + (r0 + (l & 15)) * lda + k0 + kq);
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const bf16x8 b =
          *reinterpret_cast<const bf16x8 *>(W + (nt * 16 + (l & 15)) * ldw + k0 + kq);
      acc[nt] = mfma(a, b, acc[nt]);
    }
  }
}

// The 16 x 16 tile (mt, nt) of G^T A over the block's 64 rows: G [64][ldg]
// and A [64][lda] in LDS (bf16); out[o][i] = sum_s G[s][16 mt + o] A[s][16 nt + i].
__device__ __forceinline__ f32x4 gt_times_a(const __bf16 *G, int ldg, const __bf16 *A, int lda,
                                            int mt, int nt) {
  const int l = threadIdx.x & 63;
  const int kq = (l >> 4) * 8;
  const int go = mt * 16 + (l & 15), ai = nt * 16 + (l & 15);
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int k0 = 0; k0 < 64; k0 += 32) {
    bf16x8 a, b;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      a[e] = G[(k0 + kq + e) * ldg + go];
      b[e] = A[(k0 + kq + e) * lda + ai];
    }
    acc = mfma(a, b, acc);
  }
  return acc;
}

// Column sums over the wave's 16 rows of a D tile (lanes 0..15 hold them).
__device__ __forceinline__ float column_sum16(float s) {
  s += __shfl_xor(s, 16);
  s += __shfl_xor(s, 32);
  return s;
}

// ---------------------------------------------------------------------------
// forward pass of a block of 64 normalised rows in LDS
// ---------------------------------------------------------------------------
template <int N>
struct MlpLds {
  using D = MlpDims<N>;
  __bf16 A1[64][D::KIN];   // normalised inputs
  __bf16 A2[64][D::H];     // h1
  __bf16 A3[64][D::H];     // h2
};

// Layers 1 and 2 for the wave's rows: A2, A3 (and, if given, h1, h2 in FP32).
template <int N>
__device__ __forceinline__ void hidden_layers(const MlpDev &P, MlpLds<N> &S, float (*H1)[64],
                                              float (*H2)[64]) {
  using D = MlpDims<N>;
  const int l = threadIdx.x & 63;
  const int r0 = 16 * int(threadIdx.x >> 6);
  const int rb = r0 + 4 * (l >> 4);
  {
    f32x4 acc[4] = {};
    rows_times_wt<D::KIN, 4>(&S.A1[0][0], D::KIN, P.W1, D::KIN, r0, acc);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const int c = nt * 16 + (l & 15);
      const float b = P.b1[c];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float h = tanhf(acc[nt][r] + b);
        if (H1) H1[rb + r][c] = h;
        S.A2[rb + r][c] = to_bf16(h);
      }
    }
  }
  __syncthreads();
  {
    f32x4 acc[4] = {};
    rows_times_wt<D::H, 4>(&S.A2[0][0], D::H, P.W2, D::H, r0, acc);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const int c = nt * 16 + (l & 15);
      const float b = P.b2[c];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float h = tanhf(acc[nt][r] + b);
        if (H2) H2[rb + r][c] = h;
        S.A3[rb + r][c] = to_bf16(h);
      }
    }
  }
  __syncthreads();
}

// Output layer for the wave's rows: acc[nt] = yn - b3 (add b3 per column).
template <int N>
__device__ __forceinline__ void output_layer(const MlpDev &P, MlpLds<N> &S,
                                             f32x4 (&acc)[MlpDims<N>::KOUT / 16]) {
  using D = MlpDims<N>;
  const int r0 = 16 * int(threadIdx.x >> 6);
  rows_times_wt<D::H, D::KOUT / 16>(&S.A3[0][0], D::H, P.W3, D::H, r0, acc);
}

// ---------------------------------------------------------------------------
// element features (raw, FP32) of a tile of 64 elements into F[64][NIN]
//   own: Q[v][j][i] at index v N^2 + j N + i (wave w loads variable w)
//   face f (wave w = f): the neighbour's trace at face point p, variable v
//   at index 4 N^2 + (f N + p) 4 + v; interior and periodic faces read the
//   neighbour's state and interpolate it to its face (reversed when the
//   faces run opposite), other faces use the element's own trace
// ---------------------------------------------------------------------------
template <int N>
__device__ __forceinline__ void features_tile(const DevMesh &M, const OpTables &T,
                                              const float *__restrict__ q, int tile,
                                              float (*F)[MlpDims<N>::NIN]) {
  const int l = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
  const int e0 = tile * 64 + l;
  const int e = e0 < M.E ? e0 : M.E - 1;
  const long E = M.E;
#pragma unroll
  for (int j = 0; j < N; ++j)
#pragma unroll
    for (int i = 0; i < N; ++i)
      F[l][w * N * N + j * N + i] = q[cb_index(e, (long(w) * N + j) * N + i, 4 * N * N, E)];
  // face w
  const uint32_t fw = M.face[cb_index32(uint32_t(e), uint32_t(w), 4u, uint32_t(E))];
  const int kind = face_kind_of(fw);
  const bool conf = kind == SSD_FACE_INTERIOR || kind == SSD_FACE_PERIODIC;
  const int nb = conf ? face_idx_of(fw) : e;
  const int nf = conf ? face_nf_of(fw) : w;
  const bool rev = conf && face_rev_of(fw);
  // end weights of the Lagrange basis: face at the low (0) or high (N) end
  float lo[N], hi[N];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    lo[k] = uniform(T.I[0][k]);
    hi[k] = uniform(T.I[N][k]);
  }
  const bool high = nf == 1 || nf == 2;
  const bool along_xi = nf == 0 || nf == 2;   // face parameter runs along i
#pragma unroll
  for (int v = 0; v < 4; ++v) {
#pragma unroll
    for (int p = 0; p < N; ++p) {
      float s = 0.f;
#pragma unroll
      for (int k = 0; k < N; ++k) {
        const int jj = along_xi ? k : p, ii = along_xi ? p : k;
        const float x = q[cb_index(nb, (long(v) * N + jj) * N + ii, 4 * N * N, E)];
        s += (high ? hi[k] : lo[k]) * x;
      }
      const int pp = rev ? N - 1 - p : p;
      F[l][4 * N * N + (w * N + pp) * 4 + v] = s;
    }
  }
}

// raw features of every element, rows X[e][NIN]
template <int N>
__global__ __launch_bounds__(256) void k_features(DevMesh M, OpTables T, const float *q,
                                                  float *X) {
  using D = MlpDims<N>;
  __shared__ float F[64][D::NIN];
  features_tile<N>(M, T, q, blockIdx.x, F);
  __syncthreads();
  const long base = long(blockIdx.x) * 64;
  const int rows = int(min<long>(64, M.E - base));
  for (int c = threadIdx.x; c < rows * D::NIN; c += 256)
    X[base * D::NIN + c] = F[c / D::NIN][c % D::NIN];
}

// Correction of a stage: value o = v N^2 + j N + i of element e in `add`
// (cell-blocked state layout) = scale (sig_y yn + mu_y) of the MLP of
// element e's features.
template <int N>
__global__ __launch_bounds__(256) void k_subgrid(DevMesh M, OpTables T, MlpDev P,
                                                 const float *q, float *add, float scale) {
  using D = MlpDims<N>;
  __shared__ float F[64][D::NIN];
  __shared__ MlpLds<N> S;
  features_tile<N>(M, T, q, blockIdx.x, F);
  __syncthreads();
  for (int c = threadIdx.x; c < 64 * D::KIN; c += 256) {
    const int s = c / D::KIN, i = c % D::KIN;
    const float x = i < D::NIN ? F[s][i] : 0.f;
    S.A1[s][i] = to_bf16((x - P.mu_x[i]) * P.isig_x[i]);
  }
  __syncthreads();
  hidden_layers<N>(P, S, nullptr, nullptr);
  f32x4 acc[D::KOUT / 16] = {};
  output_layer<N>(P, S, acc);
  // y through LDS (reusing F) so that each plane row is written by consecutive lanes
  float(*Y)[D::NIN] = F;
  const int l = threadIdx.x & 63;
  const int rb = 16 * int(threadIdx.x >> 6) + 4 * (l >> 4);
#pragma unroll
  for (int nt = 0; nt < D::KOUT / 16; ++nt) {
    const int o = nt * 16 + (l & 15);
    if (o < D::NOUT) {
      const float b = P.b3[o], sy = P.sig_y[o], my = P.mu_y[o];
#pragma unroll
      for (int r = 0; r < 4; ++r) Y[rb + r][o] = scale * ((acc[nt][r] + b) * sy + my);
    }
  }
  __syncthreads();
  const long e = long(blockIdx.x) * 64 + l;
  if (e < M.E)
    for (int o = int(threadIdx.x >> 6); o < D::NOUT; o += 4) add[cb_index(e, o, D::NOUT, M.E)] = Y[l][o];
}

// Y [n][NOUT] = the network of the rows X [n][NIN].
template <int N>
__global__ __launch_bounds__(256) void k_mlp_forward(MlpDev P, const float *X, long n, float *Y) {
  using D = MlpDims<N>;
  __shared__ MlpLds<N> S;
  __shared__ float Yl[64][D::KOUT];
  const long s0 = long(blockIdx.x) * 64;
  for (int c = threadIdx.x; c < 64 * D::KIN; c += 256) {
    const int s = c / D::KIN, i = c % D::KIN;
    const float x = s0 + s < n && i < D::NIN ? X[(s0 + s) * D::NIN + i] : 0.f;
    S.A1[s][i] = to_bf16((x - P.mu_x[i]) * P.isig_x[i]);
  }
  __syncthreads();
  hidden_layers<N>(P, S, nullptr, nullptr);
  f32x4 acc[D::KOUT / 16] = {};
  output_layer<N>(P, S, acc);
  const int l = threadIdx.x & 63;
  const int rb = 16 * int(threadIdx.x >> 6) + 4 * (l >> 4);
#pragma unroll
  for (int nt = 0; nt < D::KOUT / 16; ++nt) {
    const int o = nt * 16 + (l & 15);
    if (o < D::NOUT) {
      const float b = P.b3[o], sy = P.sig_y[o], my = P.mu_y[o];
#pragma unroll
      for (int r = 0; r < 4; ++r) Yl[rb + r][o] = (acc[nt][r] + b) * sy + my;
    }
  }
  __syncthreads();
  const int rows = int(min<long>(64, n - s0));
  for (int c = threadIdx.x; c < rows * D::NOUT; c += 256)
    Y[s0 * D::NOUT + c] = Yl[c / D::NOUT][c % D::NOUT];
}

// ---------------------------------------------------------------------------
// training: loss gradient of a minibatch (accumulated into the gradient
// buffers) and the Adam update
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(256) void k_mlp_grad(MlpDev P, MlpGrad G, const float *X,
                                                  const float *Tg, long n_rows, const int *idx,
                                                  int batch, float noise, uint64_t seed,
                                                  uint64_t step) {
  using D = MlpDims<N>;
  constexpr int KO = D::KOUT, H = D::H;
  __shared__ MlpLds<N> S;
  __shared__ float H1[64][64], H2[64][64];
  __shared__ float Tn[64][KO];
  __shared__ __bf16 G3[64][KO], GZ2[64][64], GZ1[64][64];
  __shared__ float red[4];
  const int l = threadIdx.x & 63;
  const int w = int(threadIdx.x >> 6);
  const int s0 = blockIdx.x * 64;
  __shared__ int rowi[64];   // sample row, -1: none (past the batch or idx out of range)
  if (threadIdx.x < 64) {
    const int s = s0 + int(threadIdx.x);
    const long r = s < batch ? long(idx[s]) : -1;
    rowi[threadIdx.x] = r >= 0 && r < n_rows ? int(r) : -1;
  }
  __syncthreads();
  for (int c = threadIdx.x; c < 64 * D::KIN; c += 256) {
    const int s = c / D::KIN, i = c % D::KIN;
    const int r = rowi[s];
    const float x = r >= 0 && i < D::NIN ? X[long(r) * D::NIN + i] : 0.f;
    float xn = (x - P.mu_x[i]) * P.isig_x[i];
    // input noise of minibatch position s0 + s, feature i, at this step
    if (noise != 0.f && r >= 0 && i < D::NIN)
      xn += noise * noise_eps(seed, (step << 32) + uint64_t(s0 + s) * D::NIN + i);
    S.A1[s][i] = to_bf16(xn);
  }
  for (int c = threadIdx.x; c < 64 * KO; c += 256) {
    const int s = c / KO, o = c % KO;
    const int r = rowi[s];
    Tn[s][o] = r >= 0 && o < D::NOUT ? (Tg[long(r) * D::NOUT + o] - P.mu_y[o]) / P.sig_y[o] : 0.f;
  }
  __syncthreads();
  hidden_layers<N>(P, S, H1, H2);
  const int rb = 16 * w + 4 * (l >> 4);
  const float gscale = 2.0f / (float(batch) * float(D::NOUT));
  float lsum = 0.f;
  {
    f32x4 acc[KO / 16] = {};
    output_layer<N>(P, S, acc);
#pragma unroll
    for (int nt = 0; nt < KO / 16; ++nt) {
      const int o = nt * 16 + (l & 15);
      const float b = o < D::NOUT ? P.b3[o] : 0.f;
      float cs = 0.f;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int s = rb + r;
        const bool ok = rowi[s] >= 0 && o < D::NOUT;
        const float d = ok ? acc[nt][r] + b - Tn[s][o] : 0.f;
        lsum += d * d;
        const float g = gscale * d;
        cs += g;
        G3[s][o] = to_bf16(g);
      }
      cs = column_sum16(cs);
      if (l < 16 && o < D::NOUT) atomicAdd(&G.b3[o], cs);
    }
  }
  __syncthreads();
  // layer 2 input gradient: gz2 = (g3 W3) (1 - h2^2)
  {
    f32x4 acc[4] = {};
    rows_times_wt<KO, 4>(&G3[0][0], KO, P.W3t, KO, 16 * w, acc);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const int c = nt * 16 + (l & 15);
      float cs = 0.f;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float h = H2[rb + r][c];
        const float g = acc[nt][r] * (1.f - h * h);
        cs += g;
        GZ2[rb + r][c] = to_bf16(g);
      }
      cs = column_sum16(cs);
      if (l < 16) atomicAdd(&G.b2[c], cs);
    }
  }
  __syncthreads();
  // layer 1 input gradient: gz1 = (gz2 W2) (1 - h1^2)
  {
    f32x4 acc[4] = {};
    rows_times_wt<H, 4>(&GZ2[0][0], H, P.W2t, H, 16 * w, acc);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const int c = nt * 16 + (l & 15);
      float cs = 0.f;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float h = H1[rb + r][c];
        const float g = acc[nt][r] * (1.f - h * h);
        cs += g;
        GZ1[rb + r][c] = to_bf16(g);
      }
      cs = column_sum16(cs);
      if (l < 16) atomicAdd(&G.b1[c], cs);
    }
  }
  __syncthreads();
  // weight gradients over the block's samples, tiles dealt to the waves
  auto store = [&](float *dst, int ld, int mt, int nt, f32x4 a) {
    const int col = nt * 16 + (l & 15);
#pragma unroll
    for (int r = 0; r < 4; ++r) atomicAdd(&dst[(mt * 16 + 4 * (l >> 4) + r) * ld + col], a[r]);
  };
  for (int t = w; t < (KO / 16) * 4; t += 4) {   // dW3 [KOUT][H]
    const int mt = t / 4, nt = t % 4;
    store(G.W3, H, mt, nt, gt_times_a(&G3[0][0], KO, &S.A3[0][0], H, mt, nt));
  }
  for (int t = w; t < 16; t += 4) {              // dW2 [H][H]
    const int mt = t / 4, nt = t % 4;
    store(G.W2, H, mt, nt, gt_times_a(&GZ2[0][0], H, &S.A2[0][0], H, mt, nt));
  }
  for (int t = w; t < 4 * (D::KIN / 16); t += 4) {   // dW1 [H][KIN]
    const int mt = t / (D::KIN / 16), nt = t % (D::KIN / 16);
    store(G.W1, D::KIN, mt, nt, gt_times_a(&GZ1[0][0], H, &S.A1[0][0], D::KIN, mt, nt));
  }
  // loss
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) lsum += __shfl_xor(lsum, o);
  if (l == 0) red[w] = lsum;
  __syncthreads();
  // the minibatch's mean loss, summed over steps on the device
  if (threadIdx.x == 0)
    atomicAdd(G.loss, double(red[0] + red[1] + red[2] + red[3]) / (double(batch) * D::NOUT));
}

// bf16 copies of flat parameter k (a weight; biases have none)
__device__ __forceinline__ void mlp_refresh(const MlpStore &S, long k, float p) {
  constexpr int H = MLP_HIDDEN;
  const __bf16 b = to_bf16(p);
  if (k < S.o_b1) {
    S.W1b[k] = b;
  } else if (k >= S.o_W2 && k < S.o_b2) {
    const long t = k - S.o_W2;
    S.W2b[t] = b;
    S.W2tb[(t % H) * H + t / H] = b;
  } else if (k >= S.o_W3 && k < S.o_b3) {
    const long t = k - S.o_W3;
    S.W3b[t] = b;
    S.W3tb[(t % H) * S.kout + t / H] = b;
  }
}

// Adam on the flat FP32 parameters; refreshes the bf16 copies and clears
// the gradients.
__global__ __launch_bounds__(256) void k_adam(MlpStore S, long n, float lr, float b1, float b2,
                                              float eps, float bc1, float bc2) {
  const long k = long(blockIdx.x) * 256 + threadIdx.x;
  if (k >= n) return;
  const float g = S.G[k];
  const float m = b1 * S.M[k] + (1.f - b1) * g;
  const float v = b2 * S.V[k] + (1.f - b2) * g * g;
  S.M[k] = m;
  S.V[k] = v;
  S.G[k] = 0.f;
  const float p = S.P[k] - lr * (m / bc1) / (sqrtf(v / bc2) + eps);
  S.P[k] = p;
  mlp_refresh(S, k, p);
}

// bf16 copies of all weights from the FP32 parameters
__global__ __launch_bounds__(256) void k_mlp_sync(MlpStore S, long n) {
  const long k = long(blockIdx.x) * 256 + threadIdx.x;
  if (k < n) mlp_refresh(S, k, S.P[k]);
}

// Per-column sums and sums of squares (FP64) of rows [n][cols] into acc.
__global__ __launch_bounds__(256) void k_moments(const float *A, long n, int cols,
                                                 double *acc) {
  const int c = threadIdx.x;
  if (c >= cols) return;
  double s = 0.0, s2 = 0.0;
  for (long r = blockIdx.x; r < n; r += gridDim.x) {
    const double x = A[r * cols + c];
    s += x;
    s2 += x * x;
  }
  atomicAdd(&acc[c], s);
  atomicAdd(&acc[cols + c], s2);
}

// ---------------------------------------------------------------------------
// restriction of a nested fine state to the coarse mesh
//   out = P qf - sub (sub may be null); rows: out[c][o] instead of the
//   cell-blocked state layout
// ---------------------------------------------------------------------------
// SPLIT: each coarse element has 4 children; otherwise the same mesh at a
// lower order (one "child", the element itself, operator r[0]).
template <int NC, int NF, bool SPLIT>
__global__ __launch_bounds__(256) void k_restrict(const float *qf, long Ef, const int *children,
                                                  long Ec, Restrict1D R, const float *sub,
                                                  float *out, int rows) {
  constexpr int NS = SPLIT ? 2 : 1;
  const long c = long(blockIdx.x) * 256 + threadIdx.x;
  if (c >= Ec) return;
  int ch[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) ch[k] = SPLIT ? children[c * 4 + k] : int(c);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    float acc[NC][NC] = {};
#pragma unroll
    for (int b = 0; b < NS; ++b)
#pragma unroll
      for (int a = 0; a < NS; ++a) {
        const long fe = ch[a + 2 * b];
#pragma unroll
        for (int jf = 0; jf < NF; ++jf) {
          float row[NC] = {};
#pragma unroll
          for (int i_f = 0; i_f < NF; ++i_f) {
            const float x = qf[cb_index(fe, (long(v) * NF + jf) * NF + i_f, 4 * NF * NF, Ef)];
#pragma unroll
            for (int ic = 0; ic < NC; ++ic) row[ic] += R.r[a][ic][i_f] * x;
          }
#pragma unroll
          for (int jc = 0; jc < NC; ++jc)
#pragma unroll
            for (int ic = 0; ic < NC; ++ic) acc[jc][ic] += R.r[b][jc][jf] * row[ic];
        }
      }
#pragma unroll
    for (int jc = 0; jc < NC; ++jc)
#pragma unroll
      for (int ic = 0; ic < NC; ++ic) {
        const long o = (long(v) * NC + jc) * NC + ic;
        float y = acc[jc][ic];
        const long co = cb_index(c, o, 4 * NC * NC, Ec);
        if (sub) y -= sub[co];
        if (rows)
          out[c * (4L * NC * NC) + o] = y;
        else
          out[co] = y;
      }
  }
}

// ---------------------------------------------------------------------------
// relaxation term of trajectory (a posteriori) training targets: rows
// T[e][o] += rate (qa - qb)[e][o], with qa and qb in the state layout
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_nudge(const float *qa, const float *qb, long E,
                                               int planes, float rate, float *T) {
  const long k = long(blockIdx.x) * 256 + threadIdx.x;
  if (k >= E * planes) return;
  const long e = k / planes, o = k - e * planes;
  const long c = cb_index(e, o, planes, E);
  T[k] += rate * (qa[c] - qb[c]);
}

hipError_t launch_nudge(const float *qa, const float *qb, long E, int planes, float rate, float *T,
                        hipStream_t s) {
  const long n = E * planes;
  if (n < 1) return hipSuccess;
  hipLaunchKernelGGL(k_nudge, dim3((n + 255) / 256), dim3(256), 0, s, qa, qb, E, planes, rate, T);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
#define SSD_MLP_DISPATCH(N, CALL)                        \
  switch (N) {                                           \
    case 2: { constexpr int NN = 2; CALL; } break;       \
    case 3: { constexpr int NN = 3; CALL; } break;       \
    case 4: { constexpr int NN = 4; CALL; } break;       \
    default: return hipErrorInvalidValue;                \
  }

hipError_t launch_features(const DevMesh &M, const OpTables &T, const float *q, float *X,
                           hipStream_t s) {
  const int grid = (M.E + 63) / 64;
  SSD_MLP_DISPATCH(M.N, hipLaunchKernelGGL(k_features<NN>, dim3(grid), dim3(256), 0, s, M, T, q,
                                           X));
  return hipGetLastError();
}

hipError_t launch_subgrid(const DevMesh &M, const OpTables &T, const MlpDev &P, const float *q,
                          float *add, float scale, hipStream_t s) {
  const int grid = (M.E + 63) / 64;
  SSD_MLP_DISPATCH(M.N, hipLaunchKernelGGL(k_subgrid<NN>, dim3(grid), dim3(256), 0, s, M, T, P,
                                           q, add, scale));
  return hipGetLastError();
}

hipError_t launch_mlp_forward(int N, const MlpDev &P, const float *X, long n, float *Y,
                              hipStream_t s) {
  if (n < 1) return hipSuccess;
  const long grid = (n + 63) / 64;
  SSD_MLP_DISPATCH(N, hipLaunchKernelGGL(k_mlp_forward<NN>, dim3(grid), dim3(256), 0, s, P, X, n,
                                         Y));
  return hipGetLastError();
}

hipError_t launch_mlp_grad(int N, const MlpDev &P, const MlpGrad &G, const float *X,
                           const float *Tg, long n_rows, const int *idx, int batch, float noise,
                           uint64_t seed, uint64_t step, hipStream_t s) {
  const int grid = (batch + 63) / 64;
  SSD_MLP_DISPATCH(N, hipLaunchKernelGGL(k_mlp_grad<NN>, dim3(grid), dim3(256), 0, s, P, G, X,
                                         Tg, n_rows, idx, batch, noise, seed, step));
  return hipGetLastError();
}

hipError_t launch_adam(const MlpStore &S, long n, float lr, float b1, float b2, float eps,
                       float bc1, float bc2, hipStream_t s) {
  const long grid = (n + 255) / 256;
  hipLaunchKernelGGL(k_adam, dim3(grid), dim3(256), 0, s, S, n, lr, b1, b2, eps, bc1, bc2);
  return hipGetLastError();
}

hipError_t launch_mlp_sync(const MlpStore &S, long n, hipStream_t s) {
  const long grid = (n + 255) / 256;
  hipLaunchKernelGGL(k_mlp_sync, dim3(grid), dim3(256), 0, s, S, n);
  return hipGetLastError();
}

hipError_t launch_moments(const float *A, long n, int cols, double *acc, hipStream_t s) {
  if (cols > 256) return hipErrorInvalidValue;
  const int grid = int(std::min<long>(std::max<long>(n, 1), 4096));
  hipLaunchKernelGGL(k_moments, dim3(grid), dim3(256), 0, s, A, n, cols, acc);
  return hipGetLastError();
}

hipError_t launch_restrict(int Nc, int Nf, const float *qf, long Ef, const int *children, long Ec,
                           const Restrict1D &R, const float *sub, float *out, bool rows,
                           hipStream_t s) {
  const long grid = (Ec + 255) / 256;
  const bool split = children != nullptr;
#define SSD_RESTRICT(NCV, NFV, SP)                                                               \
  if (Nc == NCV && Nf == NFV && split == SP) {                                                   \
    hipLaunchKernelGGL((k_restrict<NCV, NFV, SP>), dim3(grid), dim3(256), 0, s, qf, Ef,          \
                       children, Ec, R, sub, out, int(rows));                                    \
    return hipGetLastError();                                                                    \
  }
  // nested meshes
  SSD_RESTRICT(2, 2, true)
  SSD_RESTRICT(2, 4, true)
  SSD_RESTRICT(2, 6, true)
  SSD_RESTRICT(3, 3, true)
  SSD_RESTRICT(3, 4, true)
  SSD_RESTRICT(3, 5, true)
  SSD_RESTRICT(3, 6, true)
  SSD_RESTRICT(4, 6, true)
  // one mesh, lower order
  SSD_RESTRICT(2, 3, false)
  SSD_RESTRICT(2, 4, false)
  SSD_RESTRICT(2, 5, false)
  SSD_RESTRICT(2, 6, false)
  SSD_RESTRICT(3, 4, false)
  SSD_RESTRICT(3, 5, false)
  SSD_RESTRICT(3, 6, false)
  SSD_RESTRICT(4, 5, false)
  SSD_RESTRICT(4, 6, false)
  SSD_RESTRICT(5, 6, false)
#undef SSD_RESTRICT
  return hipErrorInvalidValue;
}

}  // namespace ssd

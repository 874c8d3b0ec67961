// Learned residual -> correction preconditioner for flexible GMRES.
//
// The paper's classic preconditioner is the inverse diagonal of the
// Hamiltonian (GFCC Workflow and Bottlenecks).  Here an elementwise MLP adds a
// correction to that Jacobi step.  Per element d of a complex vector r, with
// z = omega - i eta, exact diagonal D, per-system scale sD = mean|D| and
// rms n = ||r|| / sqrt(dim):
//   rh = r/n, jh = rh sD/(z + D)
//   x_d = [Re rh, Im rh, Re jh, Im jh, D/sD - 1, omega, [d < o], 100 eta]
//   y_d = W3 tanh(W2 tanh(W1 x_d + b1) + b2) + b3
//   M(r)_d = r_d/(z + D_d) + (y_d0 + i y_d1) n/sD
// Trained on (r, e) pairs with A e = r taken from the solver's own restarts
// (target t = e sD/n - jh, MSE, Adam), all in FP64 on the generic MFMA GEMM.
// Inference inside FGMRES is one fused kernel: features -> layer 1 (FMA) ->
// layer 2 on BF16 MFMA with FP32 accumulation -> layer 3 -> Jacobi + correction.
#include <algorithm>
#include <cmath>
#include <vector>

#include "ctx.h"
#include "mlp.h"

namespace gfcc {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

int64_t mlp_n_params(int W) { return int64_t(W) * MLP_F + W + int64_t(W) * W + W + 2 * W + 2; }

// offsets into the flat parameter vector
struct MlpOff {
  int64_t W1, b1, W2, b2, W3, b3;
  explicit MlpOff(int W) {
    W1 = 0;
    b1 = W1 + int64_t(W) * MLP_F;
    W2 = b1 + W;
    b2 = W2 + int64_t(W) * W;
    W3 = b2 + W;
    b3 = W3 + 2 * W;
  }
};

// counter-based sampler (splitmix64)
__device__ __forceinline__ uint64_t mix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

__device__ __forceinline__ int64_t plane_index(int64_t d, int64_t o, int64_t o_pad) {
  return d < o ? d : d - o + o_pad;
}

// features of element d (plane index pl) of vector (re, im) with rms n
__device__ __forceinline__ void feat(double re, double im, double dg, double om, double eta, double sD, double n,
                                     bool is1h, double* x) {
  const double a = re / n, b = im / n;
  const double zr = om + dg, zi = -eta;  // z + D
  const double den = sD / (zr * zr + zi * zi);
  x[0] = a;
  x[1] = b;
  x[2] = (a * zr - b * eta) * den;   // (a + ib)/(zr + i zi) = (a zr + b zi + i(b zr - a zi))/|.|^2, zi = -eta
  x[3] = (b * zr + a * eta) * den;
  x[4] = dg / sD - 1.0;
  x[5] = om;
  x[6] = is1h ? 1.0 : 0.0;
  x[7] = 100.0 * eta;
}

// ---- minibatch of (features, targets) sampled from the pair set
__global__ void mlp_sample_kernel(const double* __restrict__ R, const double* __restrict__ E, const double* omega,
                                  const double* nrm, int64_t npairs, const double* __restrict__ diag, int64_t D,
                                  int64_t o, int64_t o_pad, int64_t Dp, double eta, double sD, uint64_t seed,
                                  int64_t N, double* __restrict__ X, double* __restrict__ T) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const uint64_t h = mix64(seed ^ mix64(uint64_t(i)));
  const int64_t pi = int64_t(h % uint64_t(npairs));
  const int64_t d = int64_t(mix64(h) % uint64_t(D));
  const int64_t pl = plane_index(d, o, o_pad);
  const double* r = R + pi * 2 * Dp;
  const double* e = E + pi * 2 * Dp;
  const double n = nrm[pi];
  double x[MLP_F];
  feat(r[pl], r[Dp + pl], diag[pl], omega[pi], eta, sD, n, d < o, x);
  for (int f = 0; f < MLP_F; ++f) X[i * MLP_F + f] = x[f];
  T[i * 2 + 0] = e[pl] * sD / n - x[2];
  T[i * 2 + 1] = e[Dp + pl] * sD / n - x[3];
}

// ---- features of whole vectors (for verification)
__global__ void mlp_features_kernel(const double* __restrict__ planes, int64_t nvec, const double* omega,
                                    const double* nrm, const double* __restrict__ diag, int64_t D, int64_t o,
                                    int64_t o_pad, int64_t Dp, double eta, double sD, double* __restrict__ X) {
  const int64_t vi = blockIdx.y;
  for (int64_t d = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; d < D; d += int64_t(gridDim.x) * blockDim.x) {
    const int64_t pl = plane_index(d, o, o_pad);
    const double* r = planes + vi * 2 * Dp;
    double x[MLP_F];
    feat(r[pl], r[Dp + pl], diag[pl], omega[vi], eta, sD, nrm[vi], d < o, x);
    for (int f = 0; f < MLP_F; ++f) X[(vi * D + d) * MLP_F + f] = x[f];
  }
}

__global__ void bias_act_kernel(double* __restrict__ H, const double* __restrict__ b, int64_t N, int W, int act) {
  const int64_t n = int64_t(N) * W;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n; t += int64_t(gridDim.x) * blockDim.x) {
    const double v = H[t] + b[t % W];
    H[t] = act ? tanh(v) : v;
  }
}

// dY = 2 (Y - T) / N ; per-block partial sums of (Y - T)^2
__global__ void loss_kernel(const double* __restrict__ Y, const double* __restrict__ T, int64_t N,
                            double* __restrict__ dY, double* __restrict__ part) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < 2 * N; t += int64_t(gridDim.x) * blockDim.x) {
    const double diff = Y[t] - T[t];
    acc += diff * diff;
    dY[t] = 2.0 * diff / double(N);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void sum_kernel(const double* __restrict__ part, int n, double scale, double* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += part[i];
    out[0] = s * scale;
  }
}

__global__ void tanh_bwd_kernel(double* __restrict__ dH, const double* __restrict__ H, int64_t n) {
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n; t += int64_t(gridDim.x) * blockDim.x)
    dH[t] *= 1.0 - H[t] * H[t];
}

__global__ void adam_kernel(double* __restrict__ p, const double* __restrict__ g, double* __restrict__ m,
                            double* __restrict__ v, int64_t n, double lr, double b1, double b2, double eps,
                            double c1, double c2) {
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n; t += int64_t(gridDim.x) * blockDim.x) {
    const double gt = g[t];
    const double mt = b1 * m[t] + (1.0 - b1) * gt;
    const double vt = b2 * v[t] + (1.0 - b2) * gt * gt;
    m[t] = mt;
    v[t] = vt;
    p[t] -= lr * (mt / c1) / (sqrt(vt / c2) + eps);
  }
}

// pair errors: E[k] = Xstar[rhs[k]] - X[k]
__global__ void pair_error_kernel(double* __restrict__ E, const double* __restrict__ Xk, const double* __restrict__ Xs,
                                  const int* rhs, int64_t Dp2) {
  const int64_t k = blockIdx.y;
  const double* xs = Xs + int64_t(rhs[k]) * Dp2;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < Dp2; t += int64_t(gridDim.x) * blockDim.x)
    E[k * Dp2 + t] = xs[t] - Xk[k * Dp2 + t];
}

__global__ void to_lowp_kernel(const double* __restrict__ p, int64_t n, float* __restrict__ f32, __bf16* bf,
                               int64_t w2_off, int64_t w2_n) {
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n; t += int64_t(gridDim.x) * blockDim.x) {
    f32[t] = float(p[t]);
    if (t >= w2_off && t < w2_off + w2_n) bf[t - w2_off] = __bf16(float(p[t]));
  }
}

static unsigned nblk(int64_t n) { return unsigned(std::min<int64_t>(std::max<int64_t>((n + 255) / 256, 1), 8192)); }

// ------------------------------------------------------------------ FP64 forward / backward

void mlp_forward64(gfcc_ctx* c, int64_t N, const double* X, double* H1, double* H2, double* Y, hipStream_t s) {
  Mlp& M = *c->mlp;
  const int W = M.width;
  MlpOff off(W);
  const double* P = M.params.as<double>();
  auto lin_layer = [&](const double* A, int64_t K, const double* Wt, int64_t nout, double* C) {
    GemmArgs g;
    g.A = A;
    g.am = lin(K);
    g.B = Wt;
    g.bm = lin(K);
    g.C = C;
    g.cm = lin(nout);
    g.cn = lin(1);
    g.M = N;
    g.N = nout;
    g.K = K;
    gemm(Prec::F64, g, gemm_default_cfg(g.M, g.N, g.K), s);
  };
  lin_layer(X, MLP_F, P + off.W1, W, H1);
  hipLaunchKernelGGL(bias_act_kernel, dim3(nblk(N * W)), dim3(256), 0, s, H1, P + off.b1, N, W, 1);
  lin_layer(H1, W, P + off.W2, W, H2);
  hipLaunchKernelGGL(bias_act_kernel, dim3(nblk(N * W)), dim3(256), 0, s, H2, P + off.b2, N, W, 1);
  lin_layer(H2, W, P + off.W3, 2, Y);
  hipLaunchKernelGGL(bias_act_kernel, dim3(nblk(N * 2)), dim3(256), 0, s, Y, P + off.b3, N, 2, 0);
  GFCC_HIP(hipGetLastError());
}

// loss (device scalar) and flat gradient for a minibatch
void mlp_loss_grad64(gfcc_ctx* c, int64_t N, const double* X, const double* T, double* loss, double* grad,
                     hipStream_t s) {
  Mlp& M = *c->mlp;
  const int W = M.width;
  MlpOff off(W);
  const double* P = M.params.as<double>();
  double* H1 = M.ws.get(0, N * W, s);
  double* H2 = M.ws.get(1, N * W, s);
  double* Y = M.ws.get(2, N * 2, s);
  M.dY.ensure(size_t(N) * 2 * 8, s);
  double* dY = M.dY.as<double>();
  M.dH.ensure(size_t(N) * W * 8, s);
  M.dHT.ensure(size_t(N) * W * 8, s);
  M.ones.ensure(size_t(N) * 8, s);
  M.part.ensure(512 * 8, s);
  mlp_forward64(c, N, X, H1, H2, Y, s);
  const unsigned nb = std::min<unsigned>(512, nblk(2 * N));
  hipLaunchKernelGGL(loss_kernel, dim3(nb), dim3(256), 0, s, Y, T, N, dY, M.part.as<double>());
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(64), 0, s, M.part.as<double>(), int(nb), 1.0 / double(N), loss);
  GFCC_HIP(hipGetLastError());
  if (!M.ones_ready || M.ones_n < N) {
    std::vector<double> one(size_t(N), 1.0);
    GFCC_HIP(hipMemcpyAsync(M.ones.p, one.data(), size_t(N) * 8, hipMemcpyHostToDevice, s));
    GFCC_HIP(hipStreamSynchronize(s));
    M.ones_ready = true;
    M.ones_n = N;
  }
  // weight gradient  gW[i][j] = sum_n dZ[n][i] Hin[n][j]  (dZ^T via a transpose), bias = ones^T dZ
  auto wgrad = [&](const double* dZ, int64_t nout, const double* Hin, int64_t nin, double* gW, double* gb) {
    TView src = tview(const_cast<double*>(dZ), {N, nout});
    TView dst = tview(M.dHT.as<double>(), {nout, N});
    const int tr[2] = {1, 0};
    permute(src, tr, 1.0, dst, 0.0, s);
    GemmArgs g;
    g.A = M.dHT.p;
    g.am = lin(N);
    g.B = Hin;
    g.b_ncontig = 1;
    g.bm = lin(nin);
    g.C = gW;
    g.cm = lin(nin);
    g.cn = lin(1);
    g.M = nout;
    g.N = nin;
    g.K = N;
    gemm_auto(Prec::F64, g, M.ws, 3, s);
    GemmArgs h;
    h.A = M.ones.p;
    h.am = lin(N);
    h.B = dZ;
    h.b_ncontig = 1;
    h.bm = lin(nout);
    h.C = gb;
    h.cm = lin(nout);
    h.cn = lin(1);
    h.M = 1;
    h.N = nout;
    h.K = N;
    gemm_auto(Prec::F64, h, M.ws, 3, s);
  };
  // input gradient  dHin[n][j] = sum_i dZ[n][i] Wt[i][j]
  auto dgrad = [&](const double* dZ, int64_t nout, const double* Wt, int64_t nin, double* dHin) {
    GemmArgs g;
    g.A = dZ;
    g.am = lin(nout);
    g.B = Wt;
    g.b_ncontig = 1;
    g.bm = lin(nin);
    g.C = dHin;
    g.cm = lin(nin);
    g.cn = lin(1);
    g.M = N;
    g.N = nin;
    g.K = nout;
    gemm(Prec::F64, g, gemm_default_cfg(g.M, g.N, g.K), s);
  };
  double* dH = M.dH.as<double>();
  wgrad(dY, 2, H2, W, grad + off.W3, grad + off.b3);
  dgrad(dY, 2, P + off.W3, W, dH);
  hipLaunchKernelGGL(tanh_bwd_kernel, dim3(nblk(N * W)), dim3(256), 0, s, dH, H2, N * W);
  wgrad(dH, W, H1, W, grad + off.W2, grad + off.b2);
  // dH1 = dH2 W2 -> reuse H2's buffer (no longer needed)
  dgrad(dH, W, P + off.W2, W, H2);
  hipLaunchKernelGGL(tanh_bwd_kernel, dim3(nblk(N * W)), dim3(256), 0, s, H2, H1, N * W);
  wgrad(H2, W, X, MLP_F, grad + off.W1, grad + off.b1);
  GFCC_HIP(hipGetLastError());
}

void mlp_init(gfcc_ctx* c, int W, uint64_t seed, hipStream_t s) {
  GFCC_CHECK(W == 64 || W == 128 || W == 256, GFCC_E_ARG, "MLP width must be 64, 128 or 256");
  if (!c->mlp) c->mlp = std::make_unique<Mlp>();
  Mlp& M = *c->mlp;
  M.width = W;
  M.trained = false;
  const int64_t np = mlp_n_params(W);
  M.params.ensure(size_t(np) * 8, s);
  MlpOff off(W);
  std::vector<double> h(size_t(np), 0.0);
  // Xavier-uniform hidden layers from splitmix64, zero output layer (starts as Jacobi)
  uint64_t st = seed ^ 0x5DEECE66Dull;
  auto unif = [&]() {
    st += 0x9E3779B97F4A7C15ull;
    uint64_t x = st;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    x ^= x >> 31;
    return double(x >> 11) * (1.0 / 9007199254740992.0);
  };
  const double l1 = std::sqrt(6.0 / (MLP_F + W)), l2 = std::sqrt(6.0 / (2.0 * W));
  for (int64_t i = 0; i < int64_t(W) * MLP_F; ++i) h[off.W1 + i] = (2.0 * unif() - 1.0) * l1;
  for (int64_t i = 0; i < int64_t(W) * W; ++i) h[off.W2 + i] = (2.0 * unif() - 1.0) * l2;
  GFCC_HIP(hipMemcpyAsync(M.params.p, h.data(), size_t(np) * 8, hipMemcpyHostToDevice, s));
  M.m.ensure(size_t(np) * 8, s);
  M.v.ensure(size_t(np) * 8, s);
  GFCC_HIP(hipMemsetAsync(M.m.p, 0, size_t(np) * 8, s));
  GFCC_HIP(hipMemsetAsync(M.v.p, 0, size_t(np) * 8, s));
  GFCC_HIP(hipStreamSynchronize(s));
  M.adam_t = 0;
}

void mlp_prepare_inference(gfcc_ctx* c, hipStream_t s) {
  Mlp& M = *c->mlp;
  const int W = M.width;
  const int64_t np = mlp_n_params(W);
  MlpOff off(W);
  M.p32.ensure(size_t(np) * 4, s);
  M.w2bf.ensure(size_t(W) * W * 2, s);
  hipLaunchKernelGGL(to_lowp_kernel, dim3(nblk(np)), dim3(256), 0, s, M.params.as<double>(), np, M.p32.as<float>(),
                     M.w2bf.as<__bf16>(), off.W2, int64_t(W) * W);
  GFCC_HIP(hipGetLastError());
  M.trained = true;
}

// ------------------------------------------------------------------ fused inference

template <int W>
__global__ __launch_bounds__(256) void mlp_apply_kernel(MlpApplyArgs a) {
  constexpr int TILE = 64;
  constexpr int LDH = W + 8;
  constexpr int NF = W / 64;  // 16-column MFMA blocks per wave
  __shared__ float X[TILE][MLP_F];
  __shared__ __attribute__((aligned(16))) __bf16 H[TILE * LDH];
  __shared__ float Yo[TILE][2];
  const int q = blockIdx.y;
  const int slot = a.slots ? a.slots[q] : q;
  const double* vr = a.src + int64_t(a.src_idx ? a.src_idx[q] : q) * 2 * a.Dp;
  const double* vi = vr + a.Dp;
  const double om = a.omega[q];
  const double nrm = a.nrm ? a.nrm[q] : a.nrm_const;
  const bool use_mlp = a.mode ? (a.mode[slot] != 0) : true;
  const int tid = threadIdx.x;
  const int64_t e0 = int64_t(blockIdx.x) * TILE;
  const float* P = a.p32;
  // 1. features, Jacobi step
  double jr = 0.0, ji = 0.0;
  int64_t pl = -1;
  if (tid < TILE) {
    const int64_t d = e0 + tid;
    if (d < a.D) {
      pl = plane_index(d, a.o, a.o_pad);
      const double re = vr[pl], im = vi[pl], dg = a.diag[pl];
      double x[MLP_F];
      feat(re, im, dg, om, a.eta, a.sD, nrm, d < a.o, x);
      for (int f = 0; f < MLP_F; ++f) X[tid][f] = float(x[f]);
      const double zr = om + dg, zi = -a.eta, den = 1.0 / (zr * zr + zi * zi);
      jr = (re * zr + im * zi) * den;   // (re + i im) / (zr + i zi)
      ji = (im * zr - re * zi) * den;
    } else {
      for (int f = 0; f < MLP_F; ++f) X[tid][f] = 0.f;
    }
  }
  if (!use_mlp) {  // Jacobi fallback for this slot (uniform per block)
    if (pl >= 0) {
      a.dst[int64_t(q) * 2 * a.Dp + pl] = jr;
      a.dst[int64_t(q) * 2 * a.Dp + a.Dp + pl] = ji;
      if (a.zdst) {
        double* zz = a.zdst + a.zoff[q];
        zz[pl] = jr;
        zz[a.Dp + pl] = ji;
      }
    }
    return;
  }
  __syncthreads();
  // 2. layer 1 (K = 8) with FMAs
  for (int idx = tid; idx < TILE * W; idx += 256) {
    const int e = idx / W, w = idx % W;
    float acc = P[a.off_b1 + w];
#pragma unroll
    for (int f = 0; f < MLP_F; ++f) acc += X[e][f] * P[a.off_W1 + w * MLP_F + f];
    H[e * LDH + w] = __bf16(tanhf(acc));
  }
  __syncthreads();
  // 3. layer 2 on BF16 MFMA: rows = 64 elements, cols = W neurons split over 4 waves
  const int lane = tid & 63, wv = tid >> 6;
  v4f acc[4][NF];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < NF; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
  const int fr = lane & 15, fk = (lane >> 4) * 8;
  for (int kk = 0; kk < W; kk += 32) {
    v8bf af[4], bfr[NF];
#pragma unroll
    for (int i = 0; i < 4; ++i) af[i] = *reinterpret_cast<const v8bf*>(&H[(i * 16 + fr) * LDH + kk + fk]);
#pragma unroll
    for (int j = 0; j < NF; ++j) {
      const int n = wv * (W / 4) + j * 16 + fr;
      bfr[j] = *reinterpret_cast<const v8bf*>(&a.w2bf[int64_t(n) * W + kk + fk]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < NF; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
  }
  __syncthreads();  // every wave is done reading H1
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < NF; ++j) {
      const int n = wv * (W / 4) + j * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = i * 16 + 4 * (lane >> 4) + r;
        H[row * LDH + n] = __bf16(tanhf(acc[i][j][r] + P[a.off_b2 + n]));
      }
    }
  __syncthreads();
  // 4. layer 3 (2 outputs)
  if (tid < 2 * TILE) {
    const int e = tid >> 1, ko = tid & 1;
    float y = P[a.off_b3 + ko];
    for (int w = 0; w < W; ++w) y += float(H[e * LDH + w]) * P[a.off_W3 + ko * W + w];
    Yo[e][ko] = y;
  }
  __syncthreads();
  // 5. Jacobi + correction
  if (pl >= 0) {
    const double f = nrm / a.sD;
    const double ur = jr + double(Yo[tid][0]) * f, ui = ji + double(Yo[tid][1]) * f;
    a.dst[int64_t(q) * 2 * a.Dp + pl] = ur;
    a.dst[int64_t(q) * 2 * a.Dp + a.Dp + pl] = ui;
    if (a.zdst) {
      double* zz = a.zdst + a.zoff[q];
      zz[pl] = ur;
      zz[a.Dp + pl] = ui;
    }
  }
}

void mlp_apply(gfcc_ctx* c, MlpApplyArgs a, int64_t nvec, hipStream_t s) {
  Mlp& M = *c->mlp;
  GFCC_CHECK(M.trained, GFCC_E_STATE, "MLP preconditioner has no weights (train or set them first)");
  MlpOff off(M.width);
  a.p32 = M.p32.as<float>();
  a.w2bf = M.w2bf.as<__bf16>();
  a.off_W1 = off.W1;
  a.off_b1 = off.b1;
  a.off_b2 = off.b2;
  a.off_W3 = off.W3;
  a.off_b3 = off.b3;
  a.sD = M.sD;
  a.D = c->D;
  a.o = c->o;
  a.o_pad = c->o_pad;
  a.Dp = c->Dp;
  a.diag = c->diag.as<double>();
  dim3 grid(unsigned((c->D + 63) / 64), unsigned(nvec));
  switch (M.width) {
    case 64: hipLaunchKernelGGL(mlp_apply_kernel<64>, grid, dim3(256), 0, s, a); break;
    case 128: hipLaunchKernelGGL(mlp_apply_kernel<128>, grid, dim3(256), 0, s, a); break;
    case 256: hipLaunchKernelGGL(mlp_apply_kernel<256>, grid, dim3(256), 0, s, a); break;
    default: throw Error{GFCC_E_STATE, "bad MLP width"};
  }
  GFCC_HIP(hipGetLastError());
}

void mlp_features(gfcc_ctx* c, int64_t nvec, const double* planes, const double* omega_dev, const double* nrm_dev,
                  double eta, double* X, hipStream_t s) {
  Mlp& M = *c->mlp;
  hipLaunchKernelGGL(mlp_features_kernel, dim3(nblk(c->D), unsigned(nvec)), dim3(256), 0, s, planes, nvec, omega_dev,
                     nrm_dev, c->diag.as<double>(), c->D, c->o, c->o_pad, c->Dp, eta, M.sD, X);
  GFCC_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ training

// One Adam step (Kingma & Ba): biased moments m, v with beta1 = 0.9, beta2 = 0.999,
// bias corrections 1 - beta^t, step lr * mhat / (sqrt(vhat) + 1e-8).
void mlp_adam(gfcc_ctx* c, const double* grad, double lr, hipStream_t s) {
  Mlp& M = *c->mlp;
  const int64_t np = mlp_n_params(M.width);
  const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
  M.adam_t += 1;
  const double c1 = 1.0 - std::pow(b1, double(M.adam_t)), c2 = 1.0 - std::pow(b2, double(M.adam_t));
  hipLaunchKernelGGL(adam_kernel, dim3(nblk(np)), dim3(256), 0, s, M.params.as<double>(), grad, M.m.as<double>(),
                     M.v.as<double>(), np, lr, b1, b2, eps, c1, c2);
  GFCC_HIP(hipGetLastError());
}

void mlp_train(gfcc_ctx* c, const MlpPairs& pairs, int64_t steps, int64_t N, double lr, uint64_t seed, double eta,
               gfcc_mlp_report* rep, hipStream_t s) {
  Mlp& M = *c->mlp;
  const int64_t np = mlp_n_params(M.width);
  double* X = M.ws.get(4, N * MLP_F, s);
  double* T = M.ws.get(5, N * 2, s);
  M.grad.ensure(size_t(np) * 8, s);
  M.loss.ensure(size_t(std::max<int64_t>(steps, 1)) * 8, s);
  for (int64_t it = 0; it < steps; ++it) {
    hipLaunchKernelGGL(mlp_sample_kernel, dim3(nblk(N)), dim3(256), 0, s, pairs.R, pairs.E, pairs.omega, pairs.nrm,
                       pairs.n, c->diag.as<double>(), c->D, c->o, c->o_pad, c->Dp, eta, M.sD,
                       mix64_host(seed + 0x1000 * uint64_t(it)), N, X, T);
    mlp_loss_grad64(c, N, X, T, M.loss.as<double>() + it, M.grad.as<double>(), s);
    mlp_adam(c, M.grad.as<double>(), lr, s);
  }
  std::vector<double> L(size_t(std::max<int64_t>(steps, 1)));
  if (steps > 0)
    GFCC_HIP(hipMemcpyAsync(L.data(), M.loss.p, size_t(steps) * 8, hipMemcpyDeviceToHost, s));
  GFCC_HIP(hipStreamSynchronize(s));
  if (rep && steps > 0) {
    rep->loss_first = L[0];
    double tail = 0.0;
    const int64_t nt = std::max<int64_t>(1, steps / 20);
    for (int64_t i = steps - nt; i < steps; ++i) tail += L[size_t(i)];
    rep->loss_final = tail / double(nt);
    rep->steps = int32_t(steps);
  }
  mlp_prepare_inference(c, s);
}

void mlp_pair_errors(double* E, const double* Xk, const double* Xstar, const int* rhs_dev, int64_t npairs,
                     int64_t Dp, hipStream_t s) {
  if (npairs <= 0) return;
  hipLaunchKernelGGL(pair_error_kernel, dim3(nblk(2 * Dp), unsigned(npairs)), dim3(256), 0, s, E, Xk, Xstar, rhs_dev,
                     2 * Dp);
  GFCC_HIP(hipGetLastError());
}

}  // namespace gfcc

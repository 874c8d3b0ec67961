// Learned preconditioner: state kept in the context and kernel arguments.
#pragma once
#include <memory>

#include "gfcc_internal.h"

namespace gfcc {

constexpr int MLP_F = 8;  // features per element

struct Mlp {
  int width = 0;
  bool trained = false;
  double sD = 1.0;         // per-system scale: mean |diag(Hbar_N)|
  int64_t adam_t = 0;
  DBuf params, m, v, grad;  // FP64 master weights, Adam moments, gradient
  DBuf p32, w2bf;           // inference copies (all FP32; W2 also BF16)
  DBuf dY, dH, dHT, ones, part, loss;
  bool ones_ready = false;
  int64_t ones_n = 0;
  Scratch ws;
};

struct MlpApplyArgs {
  const double* src = nullptr;   // source vectors: 2 planes each, src + idx*2*Dp
  const int* src_idx = nullptr;  // per output vector, index into src (nullptr: identity)
  const int* slots = nullptr;    // per output vector, slot id for `mode` (nullptr: identity)
  const int* mode = nullptr;     // per slot: 1 = MLP, 0 = Jacobi fallback (nullptr: all MLP)
  const double* omega = nullptr; // per output vector
  const double* nrm = nullptr;   // per output vector rms, or nullptr: use nrm_const
  double nrm_const = 1.0;
  double eta = 0.0;
  double* dst = nullptr;         // output planes [nvec][2][Dp]
  double* zdst = nullptr;        // optional second copy (flexible GMRES Z), at zdst + zoff[q]
  const int64_t* zoff = nullptr;
  // filled by mlp_apply
  const float* p32 = nullptr;
  const __bf16* w2bf = nullptr;
  int64_t off_W1 = 0, off_b1 = 0, off_b2 = 0, off_W3 = 0, off_b3 = 0;
  double sD = 1.0;
  int64_t D = 0, o = 0, o_pad = 0, Dp = 0;
  const double* diag = nullptr;
};

struct MlpPairs {
  const double* R = nullptr;   // [n][2][Dp] residuals
  const double* E = nullptr;   // [n][2][Dp] errors (A E = R)
  const double* omega = nullptr;
  const double* nrm = nullptr; // rms of each residual
  int64_t n = 0;
};

inline uint64_t mix64_host(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

int64_t mlp_n_params(int W);
void mlp_init(struct ::gfcc_ctx* c, int W, uint64_t seed, hipStream_t s);
void mlp_prepare_inference(struct ::gfcc_ctx* c, hipStream_t s);
void mlp_forward64(struct ::gfcc_ctx* c, int64_t N, const double* X, double* H1, double* H2, double* Y, hipStream_t s);
void mlp_loss_grad64(struct ::gfcc_ctx* c, int64_t N, const double* X, const double* T, double* loss, double* grad,
                     hipStream_t s);
void mlp_apply(struct ::gfcc_ctx* c, MlpApplyArgs a, int64_t nvec, hipStream_t s);
void mlp_features(struct ::gfcc_ctx* c, int64_t nvec, const double* planes, const double* omega_dev,
                  const double* nrm_dev, double eta, double* X, hipStream_t s);
void mlp_train(struct ::gfcc_ctx* c, const MlpPairs& pairs, int64_t steps, int64_t N, double lr, uint64_t seed,
               double eta, gfcc_mlp_report* rep, hipStream_t s);
void mlp_adam(struct ::gfcc_ctx* c, const double* grad, double lr, hipStream_t s);
void mlp_pair_errors(double* E, const double* Xk, const double* Xstar, const int* rhs_dev, int64_t npairs,
                     int64_t Dp, hipStream_t s);

}  // namespace gfcc

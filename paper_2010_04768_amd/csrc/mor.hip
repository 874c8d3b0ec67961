// Model-order reduction of the X_p linear systems over frequency levels.
//
// Theory section, eq. (model): with an orthonormal basis S of m vectors,
// Hhat = S^T Hbar_N S, bhat_p = S^T b_p and chat_q = S^T c_q, the small system
// (omega - i eta + Hhat) Xhat = bhat_p gives G_qp(omega) ~ chat_q^T Xhat.
// GFCC Workflow and Bottlenecks (Algorithm 1 and eq. Lmax): an outer loop over
// levels; each level solves its (omega, p) pairs, Gram-Schmidts the solutions
// into S, projects, evaluates the model over the frequency window and picks
// the frequencies of the next level.  Level 1 takes 3 frequencies, level L > 1
// at most 2^(L-1), so there are at most log2(window / spacing) levels.
//
// Basis: real.  Re X and Im X of each solution are separate candidates, so
// Hhat is real and one projection serves every omega.  Gram-Schmidt is
// classical with one reorthogonalisation: block GEMMs against the existing
// basis, then column by column inside the new block, dropping a candidate whose
// norm falls below drop_tol times its original norm.  The projection applies
// the FP64 sigma to the new columns only and fills the new rows and columns of
// Hhat with two GEMMs.  The model solves run one workgroup per frequency: LU
// with partial pivoting of [omega - i eta + Hhat | bhat] and back substitution.
#include <algorithm>
#include <chrono>
#include <cmath>

#include "ctx.h"
#include "mor.h"

namespace gfcc {
namespace {

unsigned nblocks(int64_t n) { return unsigned(std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 2048))); }

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// out[b] = || V[b] ||  (one workgroup per vector of Dp doubles)
__global__ __launch_bounds__(256) void norms_kernel(const double* __restrict__ V, int64_t Dp, double* out) {
  __shared__ double part[4];
  const double* v = V + int64_t(blockIdx.x) * Dp;
  double s = 0.0;
  for (int64_t t = threadIdx.x; t < Dp; t += 256) s += v[t] * v[t];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = sqrt((part[0] + part[1]) + (part[2] + part[3]));
}

__global__ void scale_copy_kernel(const double* __restrict__ v, double* __restrict__ dst, int64_t Dp, double a) {
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < Dp; t += int64_t(gridDim.x) * blockDim.x)
    dst[t] = a * v[t];
}

// basis columns (plane layout) -> real vectors in the boundary layout [m][D]
__global__ void export_basis_kernel(const double* __restrict__ S, double* __restrict__ out, int64_t D, int64_t Dp,
                                    int64_t o, int64_t o_pad) {
  const int64_t b = blockIdx.y;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < D; t += int64_t(gridDim.x) * blockDim.x)
    out[b * D + t] = S[b * Dp + ((t < o) ? t : (t - o + o_pad))];
}

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cinv(double2 a) {
  const double d = 1.0 / (a.x * a.x + a.y * a.y);
  return make_double2(a.x * d, -a.y * d);
}

// One workgroup per frequency w.  A = [omega_w - i eta + Hhat | bhat] (m x (m+np)
// complex, row-major in Aw), LU with partial pivoting applied to the whole
// augmented matrix, back substitution on the np right-hand sides, then
// G[w][t] = sum_j chat[j][q] xhat[j][p] for the pairs t = (p, q) (t = p when diag).
__global__ __launch_bounds__(256) void model_kernel(const double* __restrict__ H, int ldh, int m,
                                                    const double* __restrict__ omega, double eta,
                                                    const double* __restrict__ S, int64_t Dp,
                                                    const int64_t* __restrict__ p, int np,
                                                    const double* __restrict__ Ch, int nq, int diag,
                                                    double2* __restrict__ Aw, double2* __restrict__ G,
                                                    int* __restrict__ flag) {
  __shared__ double sv[4];
  __shared__ int si[4];
  __shared__ int piv_s;
  const int w = blockIdx.x;
  const int tid = threadIdx.x;
  const int lda = m + np;
  double2* A = Aw + int64_t(w) * m * lda;
  const double wr = omega[w];
  for (int t = tid; t < m * lda; t += 256) {
    const int i = t / lda, j = t - (t / lda) * lda;
    double2 a;
    if (j < m) {
      a = make_double2(H[int64_t(i) * ldh + j], 0.0);
      if (i == j) {
        a.x += wr;
        a.y -= eta;
      }
    } else {
      a = make_double2(S[int64_t(i) * Dp + p[j - m]], 0.0);
    }
    A[t] = a;
  }
  __syncthreads();
  for (int k = 0; k < m; ++k) {
    double best = -1.0;
    int bi = k;
    for (int i = k + tid; i < m; i += 256) {
      const double2 a = A[int64_t(i) * lda + k];
      const double v = a.x * a.x + a.y * a.y;
      if (v > best) {
        best = v;
        bi = i;
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const double ob = __shfl_xor(best, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
      }
    }
    if ((tid & 63) == 0) {
      sv[tid >> 6] = best;
      si[tid >> 6] = bi;
    }
    __syncthreads();
    if (tid == 0) {
      double b = sv[0];
      int ix = si[0];
      for (int q = 1; q < 4; ++q)
        if (sv[q] > b || (sv[q] == b && si[q] < ix)) {
          b = sv[q];
          ix = si[q];
        }
      if (!(b > 0.0)) *flag = 1;
      piv_s = ix;
    }
    __syncthreads();
    const int pr = piv_s;
    if (pr != k) {
      for (int j = tid; j < lda; j += 256) {
        const double2 a = A[int64_t(k) * lda + j];
        A[int64_t(k) * lda + j] = A[int64_t(pr) * lda + j];
        A[int64_t(pr) * lda + j] = a;
      }
      __syncthreads();
    }
    double2 akk = A[int64_t(k) * lda + k];
    if (!(akk.x * akk.x + akk.y * akk.y > 0.0)) akk = make_double2(1.0, 0.0);  // singular: flagged above
    const double2 inv = cinv(akk);
    for (int i = k + 1 + tid; i < m; i += 256) A[int64_t(i) * lda + k] = cmul(A[int64_t(i) * lda + k], inv);
    __syncthreads();
    const int R = m - k - 1, Cn = lda - k - 1;
    for (int t = tid; t < R * Cn; t += 256) {
      const int ii = t / Cn;
      const int i = k + 1 + ii, j = k + 1 + (t - ii * Cn);
      const double2 l = A[int64_t(i) * lda + k], u = A[int64_t(k) * lda + j];
      double2 a = A[int64_t(i) * lda + j];
      a.x -= l.x * u.x - l.y * u.y;
      a.y -= l.x * u.y + l.y * u.x;
      A[int64_t(i) * lda + j] = a;
    }
    __syncthreads();
  }
  for (int k = m - 1; k >= 0; --k) {
    double2 ukk = A[int64_t(k) * lda + k];
    if (!(ukk.x * ukk.x + ukk.y * ukk.y > 0.0)) ukk = make_double2(1.0, 0.0);
    const double2 inv = cinv(ukk);
    for (int r = tid; r < np; r += 256) A[int64_t(k) * lda + m + r] = cmul(A[int64_t(k) * lda + m + r], inv);
    __syncthreads();
    for (int t = tid; t < k * np; t += 256) {
      const int i = t / np, r = t - (t / np) * np;
      const double2 u = A[int64_t(i) * lda + k], x = A[int64_t(k) * lda + m + r];
      double2 a = A[int64_t(i) * lda + m + r];
      a.x -= u.x * x.x - u.y * x.y;
      a.y -= u.x * x.y + u.y * x.x;
      A[int64_t(i) * lda + m + r] = a;
    }
    __syncthreads();
  }
  const int npair = diag ? np : np * nq;
  for (int t = tid; t < npair; t += 256) {
    const int pi = diag ? t : t / nq, qi = diag ? t : t - (t / nq) * nq;
    double gr = 0.0, gi = 0.0;
    for (int j = 0; j < m; ++j) {
      const double c = Ch[int64_t(j) * nq + qi];
      const double2 x = A[int64_t(j) * lda + m + pi];
      gr += c * x.x;
      gi += c * x.y;
    }
    G[int64_t(w) * npair + t] = make_double2(gr, gi);
  }
}

Mor& mor_of(gfcc_ctx* c) {
  if (!c->mor) c->mor = std::make_unique<Mor>();
  return *c->mor;
}

// Grow S, HS and H to hold `need` columns, keeping their contents.
void reserve(gfcc_ctx* c, Mor& M, int64_t need, hipStream_t s) {
  if (need <= M.cap) return;
  const int64_t Dp = c->Dp;
  const int64_t ncap = std::max<int64_t>(round_up(need, 64), 2 * M.cap);
  DBuf S2, HS2, H2;
  S2.ensure(size_t(ncap * Dp) * 8, s);
  HS2.ensure(size_t(ncap * Dp) * 8, s);
  H2.ensure(size_t(ncap * ncap) * 8, s);
  if (M.m > 0) {
    GFCC_HIP(hipMemcpyAsync(S2.p, M.S.p, size_t(M.m * Dp) * 8, hipMemcpyDeviceToDevice, s));
    GFCC_HIP(hipMemcpyAsync(HS2.p, M.HS.p, size_t(M.m * Dp) * 8, hipMemcpyDeviceToDevice, s));
    GFCC_HIP(hipMemcpy2DAsync(H2.p, size_t(ncap) * 8, M.H.p, size_t(M.cap) * 8, size_t(M.m) * 8, size_t(M.m),
                              hipMemcpyDeviceToDevice, s));
  }
  GFCC_HIP(hipStreamSynchronize(s));
  M.S = std::move(S2);
  M.HS = std::move(HS2);
  M.H = std::move(H2);
  M.cap = ncap;
}

// c[0:n] = v . S_cols[0:n]  then  v -= sum c_j S_cols[j]   (two passes)
void cgs2_block(Mor& M, int64_t k, double* V, const double* Scols, int64_t n, int64_t Dp, hipStream_t s) {
  if (n <= 0 || k <= 0) return;
  const int64_t ldc = round_up(n, 8);
  M.coef.ensure(size_t(k * ldc) * 8, s);
  double* C = M.coef.as<double>();
  for (int pass = 0; pass < 2; ++pass) {
    GemmArgs g;
    g.A = V;
    g.am = lin(Dp);
    g.B = Scols;
    g.bm = lin(Dp);
    g.M = k;
    g.N = n;
    g.K = Dp;
    g.C = C;
    g.cm = lin(ldc);
    g.cn = lin(1);
    gemm_auto(Prec::F64, g, M.scr, 0, s);
    GemmArgs u;
    u.A = C;
    u.am = lin(ldc);
    u.B = Scols;
    u.bm = lin(Dp);
    u.b_ncontig = 1;
    u.M = k;
    u.N = Dp;
    u.K = n;
    u.C = V;
    u.cm = lin(Dp);
    u.cn = lin(1);
    u.alpha = -1.0;
    u.beta = 1.0;
    gemm(Prec::F64, u, gemm_default_cfg(k, Dp, n), s);
  }
}

}  // namespace

void mor_reset(gfcc_ctx* c) { mor_of(c).m = 0; }

int64_t mor_size(gfcc_ctx* c) { return c->mor ? c->mor->m : 0; }

// Append the orthonormalised Re/Im parts of nb complex vectors (boundary layout,
// device) to the basis and extend Hhat.  Returns the number of columns added.
int64_t mor_extend(gfcc_ctx* c, int64_t nb, const double* X, double drop_tol, hipStream_t s, double* t_basis,
                   double* t_project) {
  Mor& M = mor_of(c);
  const int64_t Dp = c->Dp, k = 2 * nb, m0 = M.m;
  if (nb <= 0) return 0;
  const double t0 = now_s();
  reserve(c, M, m0 + k, s);
  M.V.ensure(size_t(k * Dp) * 8, s);
  M.nrm.ensure(size_t(k + 1) * 8, s);
  double* V = M.V.as<double>();
  double* S = M.S.as<double>();
  to_planes(c, nb, X, V, s);
  hipLaunchKernelGGL(norms_kernel, dim3(unsigned(k)), dim3(256), 0, s, V, Dp, M.nrm.as<double>());
  GFCC_HIP(hipGetLastError());
  std::vector<double> n0(static_cast<size_t>(k));
  GFCC_HIP(hipMemcpyAsync(n0.data(), M.nrm.p, size_t(k) * 8, hipMemcpyDeviceToHost, s));
  cgs2_block(M, k, V, S, m0, Dp, s);
  GFCC_HIP(hipStreamSynchronize(s));
  int64_t acc = 0;
  for (int64_t j = 0; j < k; ++j) {
    if (!(n0[size_t(j)] > 0.0)) continue;
    double* v = V + j * Dp;
    cgs2_block(M, 1, v, S + m0 * Dp, acc, Dp, s);
    hipLaunchKernelGGL(norms_kernel, dim3(1), dim3(256), 0, s, v, Dp, M.nrm.as<double>() + k);
    GFCC_HIP(hipGetLastError());
    double n1 = 0.0;
    GFCC_HIP(hipMemcpyAsync(&n1, M.nrm.as<double>() + k, 8, hipMemcpyDeviceToHost, s));
    GFCC_HIP(hipStreamSynchronize(s));
    GFCC_CHECK(std::isfinite(n1), GFCC_E_STATE, "non-finite vector in the model basis");
    if (n1 <= drop_tol * n0[size_t(j)]) continue;
    hipLaunchKernelGGL(scale_copy_kernel, dim3(nblocks(Dp)), dim3(256), 0, s, v, S + (m0 + acc) * Dp, Dp, 1.0 / n1);
    GFCC_HIP(hipGetLastError());
    ++acc;
  }
  M.m = m0 + acc;
  GFCC_HIP(hipStreamSynchronize(s));
  const double t1 = now_s();
  if (acc > 0) {
    double* HS = M.HS.as<double>();
    double* H = M.H.as<double>();
    sigma_planes(c, acc, S + m0 * Dp, HS + m0 * Dp, GFCC_FP64, s);
    GemmArgs g;  // new columns: Hhat[0:m][m0:m] = S[0:m] . HS[m0:m]
    g.A = S;
    g.am = lin(Dp);
    g.B = HS + m0 * Dp;
    g.bm = lin(Dp);
    g.M = M.m;
    g.N = acc;
    g.K = Dp;
    g.C = H + m0;
    g.cm = lin(M.cap);
    g.cn = lin(1);
    gemm_auto(Prec::F64, g, M.scr, 0, s);
    if (m0 > 0) {  // new rows: Hhat[m0:m][0:m0] = S[m0:m] . HS[0:m0]
      GemmArgs r;
      r.A = S + m0 * Dp;
      r.am = lin(Dp);
      r.B = HS;
      r.bm = lin(Dp);
      r.M = acc;
      r.N = m0;
      r.K = Dp;
      r.C = H + m0 * M.cap;
      r.cm = lin(M.cap);
      r.cn = lin(1);
      gemm_auto(Prec::F64, r, M.scr, 0, s);
    }
    GFCC_HIP(hipStreamSynchronize(s));
  }
  const double t2 = now_s();
  if (t_basis) *t_basis += t1 - t0;
  if (t_project) *t_project += t2 - t1;
  return acc;
}

// Model G on the frequencies w[0:nw]: G[w][p][q] (diag: G[w][p] with q = p),
// complex interleaved, device.
void mor_model(gfcc_ctx* c, int64_t np, const int64_t* p, int64_t nq, const int64_t* q, bool diag, int64_t nw,
               const double* w, double eta, double* G, hipStream_t s) {
  Mor& M = mor_of(c);
  GFCC_CHECK(M.m > 0, GFCC_E_STATE, "the model basis is empty");
  if (diag) {
    q = p;
    nq = np;
  }
  const int64_t m = M.m, Dp = c->Dp;
  GFCC_CHECK(m * (m + np) < (int64_t(1) << 31) && M.cap < (int64_t(1) << 31), GFCC_E_ARG, "model too large");
  M.pdev.ensure(size_t(np + nq + nw) * 8, s);
  int64_t* pd = M.pdev.as<int64_t>();
  double* wd = M.pdev.as<double>() + np + nq;
  GFCC_HIP(hipMemcpyAsync(pd, p, size_t(np) * 8, hipMemcpyHostToDevice, s));
  GFCC_HIP(hipMemcpyAsync(pd + np, q, size_t(nq) * 8, hipMemcpyHostToDevice, s));
  GFCC_HIP(hipMemcpyAsync(wd, w, size_t(nw) * 8, hipMemcpyHostToDevice, s));
  M.rows.ensure(size_t(nq * Dp) * 8, s);
  make_left_rows(c, nq, pd + np, M.rows.as<double>(), s);
  M.Ch.ensure(size_t(m * nq) * 8, s);
  GemmArgs g;  // chat[j][k] = s_j . c_{q_k}
  g.A = M.S.p;
  g.am = lin(Dp);
  g.B = M.rows.p;
  g.bm = lin(Dp);
  g.M = m;
  g.N = nq;
  g.K = Dp;
  g.C = M.Ch.as<double>();
  g.cm = lin(nq);
  g.cn = lin(1);
  gemm_auto(Prec::F64, g, M.scr, 0, s);
  M.flag.ensure(8, s);
  GFCC_HIP(hipMemsetAsync(M.flag.p, 0, 8, s));
  const int64_t per_w = m * (m + np) * 16;
  const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(nw, (int64_t(2) << 30) / per_w));
  M.Aw.ensure(size_t(chunk * per_w), s);
  const int64_t npair = diag ? np : np * nq;
  for (int64_t w0 = 0; w0 < nw; w0 += chunk) {
    const int64_t cnt = std::min(chunk, nw - w0);
    hipLaunchKernelGGL(model_kernel, dim3(unsigned(cnt)), dim3(256), 0, s, M.H.as<double>(), int(M.cap), int(m),
                       wd + w0, eta, M.S.as<double>(), Dp, pd, int(np), M.Ch.as<double>(), int(nq), diag ? 1 : 0,
                       M.Aw.as<double2>(), reinterpret_cast<double2*>(G) + w0 * npair, M.flag.as<int>());
    GFCC_HIP(hipGetLastError());
  }
  int flag = 0;
  GFCC_HIP(hipMemcpyAsync(&flag, M.flag.p, 4, hipMemcpyDeviceToHost, s));
  GFCC_HIP(hipStreamSynchronize(s));
  GFCC_CHECK(flag == 0, GFCC_E_STATE, "singular model system");
}

void mor_export(gfcc_ctx* c, int which, double* dst, hipStream_t s) {
  Mor& M = mor_of(c);
  if (M.m == 0) return;
  if (which == 0) {  // Hhat [m][m]
    GFCC_HIP(hipMemcpy2DAsync(dst, size_t(M.m) * 8, M.H.p, size_t(M.cap) * 8, size_t(M.m) * 8, size_t(M.m),
                              hipMemcpyDeviceToDevice, s));
  } else {  // S [m][D]
    hipLaunchKernelGGL(export_basis_kernel, dim3(nblocks(c->D), unsigned(M.m)), dim3(256), 0, s, M.S.as<double>(),
                       dst, c->D, c->Dp, c->n1, c->p1);
    GFCC_HIP(hipGetLastError());
  }
}

// The level loop over a uniform ascending grid w[0:nw].
void mor_greens(gfcc_ctx* c, int64_t np, const int64_t* p, int64_t nw, const double* w, double eta,
                const gfcc_mor_opts* o, double* G, int32_t* level_of, gfcc_mor_report* rep, hipStream_t s,
                bool* all_converged) {
  Mor& M = mor_of(c);
  gfcc_mor_report r{};
  std::vector<int32_t> lev(static_cast<size_t>(nw), 0);
  int lmax = 1;
  if (nw >= 3) {
    const double dw = (w[nw - 1] - w[0]) / double(nw - 1);
    lmax = std::max(1, int(std::floor(std::log2((w[nw - 1] - w[0]) / dw) + 1e-9)));
  }
  if (o->max_levels > 0) lmax = std::min(lmax, int(o->max_levels));
  mor_reset(c);
  DBuf Xs, Gs;
  std::map<int64_t, std::vector<double>> direct;  // grid index -> G_pp (re, im) per p

  auto solve_points = [&](const std::vector<int64_t>& idx) {
    const int64_t nr = int64_t(idx.size()) * np;
    std::vector<int64_t> P(static_cast<size_t>(nr));
    std::vector<double> W(static_cast<size_t>(nr));
    for (int64_t t = 0; t < nr; ++t) {
      P[size_t(t)] = p[t % np];
      W[size_t(t)] = w[idx[size_t(t / np)]];
    }
    Xs.ensure(size_t(nr * c->D) * 16, s);
    Gs.ensure(size_t(nr) * 16, s);
    std::vector<gfcc_rhs_info> info(static_cast<size_t>(nr));
    bool conv = true;
    const double t0 = now_s();
    gfcc_solve_opts so = o->solve;
    so.checkpoint = nullptr;  // the level loop's own solves are not resumable rows of a request
    solve_batch(c, nr, P.data(), W.data(), eta, 1, nullptr, &so, Gs.as<double>(), Xs.as<double>(), info.data(),
                s, &conv, nullptr);
    std::vector<double> g(static_cast<size_t>(2 * nr));
    GFCC_HIP(hipMemcpyAsync(g.data(), Gs.p, size_t(nr) * 16, hipMemcpyDeviceToHost, s));
    GFCC_HIP(hipStreamSynchronize(s));
    r.t_solve += now_s() - t0;
    if (!conv) *all_converged = false;
    for (size_t k = 0; k < idx.size(); ++k)
      direct[idx[k]] = std::vector<double>(g.begin() + int64_t(k) * 2 * np, g.begin() + int64_t(k + 1) * 2 * np);
    r.n_solved += int32_t(idx.size());
    mor_extend(c, nr, Xs.as<double>(), o->drop_tol, s, &r.t_basis, &r.t_project);
  };

  std::vector<std::pair<int64_t, int64_t>> open;
  {
    std::vector<int64_t> todo;
    if (nw < 3) {
      for (int64_t k = 0; k < nw; ++k) todo.push_back(k);
    } else {
      const int64_t mid = (nw - 1) / 2;
      todo = {0, mid, nw - 1};
      if (mid > 1) open.push_back({0, mid});
      if (nw - 1 - mid > 1) open.push_back({mid, nw - 1});
    }
    for (int64_t k : todo) lev[size_t(k)] = 1;
    r.per_level[0] = int32_t(todo.size());
    solve_points(todo);
  }
  int level = 1;
  double last_err = 0.0;
  DBuf Gm;
  while (!open.empty() && level < lmax) {
    ++level;
    std::vector<int64_t> mids;
    for (auto& iv : open) mids.push_back((iv.first + iv.second) / 2);
    std::vector<int64_t> todo = mids;
    std::sort(todo.begin(), todo.end());
    todo.erase(std::unique(todo.begin(), todo.end()), todo.end());
    std::vector<double> wt(todo.size());
    for (size_t k = 0; k < todo.size(); ++k) wt[k] = w[todo[k]];
    // predict with the model built so far, then solve directly
    Gm.ensure(size_t(todo.size() * np) * 16, s);
    const double tm = now_s();
    mor_model(c, np, p, np, p, true, int64_t(todo.size()), wt.data(), eta, Gm.as<double>(), s);
    std::vector<double> gm(size_t(2 * np) * todo.size());
    GFCC_HIP(hipMemcpyAsync(gm.data(), Gm.p, gm.size() * 8, hipMemcpyDeviceToHost, s));
    GFCC_HIP(hipStreamSynchronize(s));
    r.t_model += now_s() - tm;
    for (int64_t k : todo) lev[size_t(k)] = level;
    if (level <= 16) r.per_level[level - 1] = int32_t(todo.size());
    solve_points(todo);
    std::map<int64_t, double> err;
    last_err = 0.0;
    for (size_t k = 0; k < todo.size(); ++k) {
      const std::vector<double>& d = direct[todo[k]];
      double e = 0.0;
      for (int64_t i = 0; i < np; ++i) {
        const double dr = gm[(k * np + i) * 2] - d[size_t(2 * i)], di = gm[(k * np + i) * 2 + 1] - d[size_t(2 * i + 1)];
        const double den = std::hypot(d[size_t(2 * i)], d[size_t(2 * i + 1)]);
        e = std::max(e, std::hypot(dr, di) / den);
      }
      err[todo[k]] = e;
      last_err = std::max(last_err, e);
    }
    std::vector<std::pair<int64_t, int64_t>> nxt;
    for (size_t k = 0; k < open.size(); ++k) {
      const int64_t a = open[k].first, b = open[k].second, cm = mids[k];
      if (err[cm] > o->tol) {
        if (cm - a > 1) nxt.push_back({a, cm});
        if (b - cm > 1) nxt.push_back({cm, b});
      }
    }
    open.swap(nxt);
  }
  const double tm = now_s();
  mor_model(c, np, p, np, p, true, nw, w, eta, G, s);
  r.t_model += now_s() - tm;
  r.levels = level;
  r.m = int32_t(M.m);
  r.converged = open.empty() ? 1 : 0;
  r.max_mid_err = last_err;
  if (rep) *rep = r;
  if (level_of) std::copy(lev.begin(), lev.end(), level_of);
}

}  // namespace gfcc

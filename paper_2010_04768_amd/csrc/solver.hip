// Batched restarted GMRES / flexible GMRES for (omega + Hbar_N - i eta) X_p = b_p
// (paper, GFCC Workflow and Bottlenecks: GMRES, minimal residual, non-increasing residual; the inverse
// diagonal of the Hamiltonian as the classic preconditioner).
//
// A persistent window of `batch` slots holds one right-hand side each.  Every
// inner iteration advances all active slots by one Arnoldi step with a single
// batched sigma product; slots sit at different Krylov steps, so every kernel
// reads its slot's own step counter.  When a slot's cycle ends (residual
// estimate below its cycle tolerance, restart length reached or max_iter) the
// host gathers those slots, forms X, recomputes the true residual with an FP64
// sigma, and either restarts the slot, or finishes it -- G_qp = c_q^T X is
// formed right away and the slot is refilled from the queue of (p, omega)
// pairs (the paper's dynamic pickup of the next orbital by an idle process
// group, Implementation Details, here at slot granularity).
//
// Orthogonalisation is classical Gram-Schmidt applied twice (CGS2), FP64,
// with the complex inner product <u, w> = sum conj(u) w.  The second
// projection's coefficients come from the Gram matrix of the basis:
// V^H (w - V h1) = h1 - G h1 with G = V^H V, so one pass over the basis forms
// h1 = V^H w together with the new column of G (<V_j, V_k>), and a second pass
// forms w - V (2 h1 - G h1) and its norm -- the same projections as
// re-reading the basis for an explicit second pass, two reads of it instead
// of four.  Givens rotations as
// in the oracle.  In GMRES-IR mode (FP32/BF16 sigma) the inner cycle stops at
// a tolerance relative to the cycle's starting residual that the reduced
// precision operator can deliver; the restart's FP64 true residual drives the
// refinement.
#include <unistd.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <set>
#include <string>
#include <vector>

#include "ctx.h"

namespace gfcc {

struct cplx {
  double re, im;
};

constexpr int VT = 256;         // threads per vector-kernel block
constexpr int VE = 8;           // elements per thread
constexpr int CH = VT * VE;     // elements per chunk
constexpr int MAXM = 64;        // maximum restart length
constexpr int PS = 2 * (MAXM + 1);  // partial-dot stride per chunk

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
  return x;
}

struct SolverDev {
  double* V;       // [B][m+1][2][Dp]
  double* Z;       // [B][m][2][Dp]  (flexible only)
  double* X;       // [B][2][Dp]
  cplx* H;         // [B][m][m+1]   H[s][k][j] = H(j, k)
  cplx* cs;        // [B][m]
  cplx* sn;        // [B][m]
  cplx* g;         // [B][m+1]
  cplx* y;         // [B][m]
  cplx* z;         // [B]  omega - i eta
  int* kk;         // [B]  current Krylov step
  double* ctol;    // [B]  cycle tolerance (absolute)
  double* res;     // [B]  residual estimate |g_{k+1}|
  int* flag;       // [B]  0 while the cycle runs; 1 done, 3 non-finite: the slot's kernels skip it
  int* fresh;      // [B]  1 in the iteration whose Givens step stopped the cycle (its scaling still runs)
  cplx* part;      // [na][nch][PS] partial dots: <V_j, w> at j, <V_j, V_k> at MAXM+1+j
  cplx* Gm;        // [B][m][m+1]   Gm[s][k][j] = <V_j, V_k>, j <= k
  cplx* h;         // [na][MAXM+1]
  double* npart;   // [na][nch]
  double* norm;    // [na]
  int m;
  int64_t Dp;
  int nch;
};

__device__ __forceinline__ double* vec(const SolverDev& d, int s, int j, int c) {
  return d.V + ((int64_t(s) * (d.m + 1) + j) * 2 + c) * d.Dp;
}

// ---- new right-hand sides: V0 = b / |b|, X = 0, g = (|b|, 0, ...), k = 0.
// b = e_p when brow[q] < 0 (occupied p), else row brow[q] of `brows`.
__global__ void init_slots_kernel(SolverDev d, const int* slots, const int* ps, const int* brow,
                                  const double* brows, const double* bnorm, const cplx* zs, const double* ctol,
                                  int n) {
  const int q = blockIdx.y;
  if (q >= n) return;
  const int s = slots[q];
  const int br = brow[q];
  const double bn = br < 0 ? 1.0 : bnorm[br];
  const double* b = br < 0 ? nullptr : brows + int64_t(br) * d.Dp;
  const int64_t i0 = int64_t(blockIdx.x) * CH;
  for (int c = 0; c < 2; ++c) {
    double* v0 = vec(d, s, 0, c);
    double* x = d.X + (int64_t(s) * 2 + c) * d.Dp;
    for (int e = threadIdx.x; e < CH; e += VT) {
      const int64_t t = i0 + e;
      if (t < d.Dp) {
        double val = 0.0;
        if (c == 0) val = b ? b[t] / bn : (t == ps[q] ? 1.0 : 0.0);
        v0[t] = val;
        x[t] = 0.0;
      }
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    d.kk[s] = 0;
    d.z[s] = zs[q];
    d.ctol[s] = ctol[q];
    d.res[s] = bn;
    d.flag[s] = 0;
    d.fresh[s] = 0;
    for (int j = 0; j <= d.m; ++j) d.g[int64_t(s) * (d.m + 1) + j] = cplx{j == 0 ? bn : 0.0, 0.0};
  }
}

// ---- preconditioner: u = M^-1 V[k]  into the dense sigma input planes
__global__ void precond_kernel(SolverDev d, const int* act, double* win, const double* diag, int mode, int flex) {
  const int q = blockIdx.y;
  const int s = act[q];
  if (d.flag[s] != 0) return;  // cycle stopped earlier in this run of iterations
  const int k = d.kk[s];
  const cplx z = d.z[s];
  const double* vr = vec(d, s, k, 0);
  const double* vi = vec(d, s, k, 1);
  double* ur = win + (int64_t(q) * 2) * d.Dp;
  double* ui = ur + d.Dp;
  double* zr = flex ? d.Z + ((int64_t(s) * d.m + k) * 2) * d.Dp : nullptr;
  const int64_t i0 = int64_t(blockIdx.x) * CH;
  for (int e = threadIdx.x; e < CH; e += VT) {
    const int64_t t = i0 + e;
    if (t >= d.Dp) break;
    double a = vr[t], b = vi[t];
    if (mode == GFCC_PC_JACOBI) {
      const double dr = z.re + diag[t], di = z.im;
      const double den = 1.0 / (dr * dr + di * di);
      const double nr = (a * dr + b * di) * den, ni = (b * dr - a * di) * den;
      a = nr;
      b = ni;
    }
    ur[t] = a;
    ui[t] = b;
    if (zr) {
      zr[t] = a;
      zr[d.Dp + t] = b;
    }
  }
}

// pass 0: w = z u + sigma -> V[k+1]; partial <V_j, w> and <V_j, V_k>, j <= k
// pass 2: w -= sum_j h_j V_j (in place); partial ||w||^2
__global__ __launch_bounds__(VT) void arnoldi_kernel(SolverDev d, const int* act, const double* win,
                                                     const double* wout, int pass) {
  const int q = blockIdx.y;
  const int s = act[q];
  if (d.flag[s] != 0) return;
  const int k = d.kk[s];
  const int64_t i0 = int64_t(blockIdx.x) * CH;
  double* wr = vec(d, s, k + 1, 0);
  double* wi = vec(d, s, k + 1, 1);
  double xr[VE], xi[VE];
  if (pass == 0) {
    const cplx z = d.z[s];
    const double* ur = win + (int64_t(q) * 2) * d.Dp;
    const double* sr = wout + (int64_t(q) * 2) * d.Dp;
#pragma unroll
    for (int e = 0; e < VE; ++e) {
      const int64_t t = i0 + threadIdx.x + e * VT;
      if (t < d.Dp) {
        const double a = ur[t], b = ur[d.Dp + t];
        xr[e] = z.re * a - z.im * b + sr[t];
        xi[e] = z.re * b + z.im * a + sr[d.Dp + t];
        wr[t] = xr[e];
        wi[t] = xi[e];
      } else {
        xr[e] = xi[e] = 0.0;
      }
    }
  } else {
    const cplx* h = d.h + int64_t(q) * (MAXM + 1);
#pragma unroll
    for (int e = 0; e < VE; ++e) {
      const int64_t t = i0 + threadIdx.x + e * VT;
      xr[e] = (t < d.Dp) ? wr[t] : 0.0;
      xi[e] = (t < d.Dp) ? wi[t] : 0.0;
    }
    for (int j = 0; j <= k; ++j) {
      const cplx hj = h[j];
      const double* vr = vec(d, s, j, 0);
      const double* vi = vec(d, s, j, 1);
#pragma unroll
      for (int e = 0; e < VE; ++e) {
        const int64_t t = i0 + threadIdx.x + e * VT;
        if (t < d.Dp) {
          const double a = vr[t], b = vi[t];
          xr[e] -= hj.re * a - hj.im * b;
          xi[e] -= hj.re * b + hj.im * a;
        }
      }
    }
    double acc = 0.0;
#pragma unroll
    for (int e = 0; e < VE; ++e) {
      const int64_t t = i0 + threadIdx.x + e * VT;
      if (t < d.Dp) {
        wr[t] = xr[e];
        wi[t] = xi[e];
      }
      acc += xr[e] * xr[e] + xi[e] * xi[e];
    }
    __shared__ double red[VT / 64];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0;
      for (int w = 0; w < VT / 64; ++w) t += red[w];
      d.npart[int64_t(q) * d.nch + blockIdx.x] = t;
    }
    return;
  }
  // pass 0: dots with every basis vector of w and of V_k
  double kr[VE], ki[VE];
  {
    const double* vr = vec(d, s, k, 0);
    const double* vi = vec(d, s, k, 1);
#pragma unroll
    for (int e = 0; e < VE; ++e) {
      const int64_t t = i0 + threadIdx.x + e * VT;
      kr[e] = (t < d.Dp) ? vr[t] : 0.0;
      ki[e] = (t < d.Dp) ? vi[t] : 0.0;
    }
  }
  __shared__ double lds[VT / 64][MAXM + 1][4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int j = 0; j <= k; ++j) {
    const double* vr = vec(d, s, j, 0);
    const double* vi = vec(d, s, j, 1);
    double a = 0.0, b = 0.0, ga = 0.0, gb = 0.0;
#pragma unroll
    for (int e = 0; e < VE; ++e) {
      const int64_t t = i0 + threadIdx.x + e * VT;
      if (t < d.Dp) {
        const double ur = vr[t], ui = vi[t];
        a += ur * xr[e] + ui * xi[e];  // conj(v) w
        b += ur * xi[e] - ui * xr[e];
        ga += ur * kr[e] + ui * ki[e];  // conj(v) V_k
        gb += ur * ki[e] - ui * kr[e];
      }
    }
    a = wave_sum(a);
    b = wave_sum(b);
    ga = wave_sum(ga);
    gb = wave_sum(gb);
    if (lane == 0) {
      lds[wv][j][0] = a;
      lds[wv][j][1] = b;
      lds[wv][j][2] = ga;
      lds[wv][j][3] = gb;
    }
  }
  __syncthreads();
  if (int(threadIdx.x) <= k) {
    double a = 0, b = 0, ga = 0, gb = 0;
    for (int w = 0; w < VT / 64; ++w) {
      a += lds[w][threadIdx.x][0];
      b += lds[w][threadIdx.x][1];
      ga += lds[w][threadIdx.x][2];
      gb += lds[w][threadIdx.x][3];
    }
    cplx* pp = d.part + (int64_t(q) * d.nch + blockIdx.x) * PS;
    pp[threadIdx.x] = cplx{a, b};
    pp[MAXM + 1 + threadIdx.x] = cplx{ga, gb};
  }
}

// Per slot: h1 = sum of the chunk partials of <V_j, w>, the new Gram column
// G(j, k) = <V_j, V_k>, then h = h1 + (h1 - G h1) -> d.h and H(:, k).
__global__ void reduce_hg_kernel(SolverDev d, const int* act) {
  const int q = blockIdx.x;
  const int s = act[q];
  if (d.flag[s] != 0) return;
  const int k = d.kk[s];
  const int m = d.m;
  const int j = threadIdx.x;
  __shared__ cplx h1[MAXM + 1];
  cplx* Gk = d.Gm + (int64_t(s) * m + k) * (m + 1);
  if (j <= k) {
    double a = 0, b = 0, ga = 0, gb = 0;
    for (int c = 0; c < d.nch; ++c) {
      const cplx* pp = d.part + (int64_t(q) * d.nch + c) * PS;
      a += pp[j].re;
      b += pp[j].im;
      ga += pp[MAXM + 1 + j].re;
      gb += pp[MAXM + 1 + j].im;
    }
    h1[j] = cplx{a, b};
    Gk[j] = cplx{ga, gb};
  }
  __syncthreads();
  if (j > k) return;
  // (G h1)_j = sum_i G(j, i) h1_i; column i of Gm holds G(0..i, i); G(j, i) = conj(G(i, j))
  double gr = 0.0, gi = 0.0;
  for (int i = 0; i <= k; ++i) {
    cplx gji;
    if (j <= i) {
      gji = d.Gm[(int64_t(s) * m + i) * (m + 1) + j];
    } else {
      const cplx gij = d.Gm[(int64_t(s) * m + j) * (m + 1) + i];
      gji = cplx{gij.re, -gij.im};
    }
    gr += gji.re * h1[i].re - gji.im * h1[i].im;
    gi += gji.re * h1[i].im + gji.im * h1[i].re;
  }
  const cplx h = cplx{2.0 * h1[j].re - gr, 2.0 * h1[j].im - gi};
  d.h[int64_t(q) * (MAXM + 1) + j] = h;
  d.H[(int64_t(s) * m + k) * (m + 1) + j] = h;
}

// ||w||, H(k+1, k), Givens rotation, residual estimate, cycle flag
// stat (window size B): flags at [0, B), Krylov steps at [B, 2B), residual estimates as doubles from
// int offset 2B, each indexed by the position in the active list.  A slot whose cycle stopped in an
// earlier iteration only reports its state.
__global__ void givens_kernel(SolverDev d, const int* act, int* stat, int B, int iters_left_any) {
  const int q = blockIdx.x;
  const int s = act[q];
  int* flags_out = stat;
  int* k_out = stat + B;
  double* res_out = reinterpret_cast<double*>(stat + 2 * B);
  if (d.flag[s] != 0) {
    if (threadIdx.x == 0) {
      d.fresh[s] = 0;
      flags_out[q] = d.flag[s];
      k_out[q] = d.kk[s];
      res_out[q] = d.res[s];
    }
    return;
  }
  __shared__ double red[64];
  double acc = 0.0;
  for (int c = threadIdx.x; c < d.nch; c += 64) acc += d.npart[int64_t(q) * d.nch + c];
  red[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x != 0) return;
  double nrm2 = 0.0;
  for (int t = 0; t < 64; ++t) nrm2 += red[t];
  const double nrm = sqrt(nrm2);
  const int k = d.kk[s];
  const int m = d.m;
  cplx* Hc = d.H + (int64_t(s) * m + k) * (m + 1);
  Hc[k + 1] = cplx{nrm, 0.0};
  cplx* cs = d.cs + int64_t(s) * m;
  cplx* sn = d.sn + int64_t(s) * m;
  cplx* g = d.g + int64_t(s) * (m + 1);
  for (int j = 0; j < k; ++j) {  // previous rotations
    const cplx hj = Hc[j], hj1 = Hc[j + 1];
    const cplx c = cs[j], sj = sn[j];
    // [h_j; h_j1] <- [conj(c) h_j + conj(s) h_j1; -s h_j + c h_j1]
    Hc[j] = cplx{c.re * hj.re + c.im * hj.im + sj.re * hj1.re + sj.im * hj1.im,
                 c.re * hj.im - c.im * hj.re + sj.re * hj1.im - sj.im * hj1.re};
    Hc[j + 1] = cplx{-(sj.re * hj.re - sj.im * hj.im) + (c.re * hj1.re - c.im * hj1.im),
                     -(sj.re * hj.im + sj.im * hj.re) + (c.re * hj1.im + c.im * hj1.re)};
  }
  const cplx a = Hc[k];
  const double bb = Hc[k + 1].re;  // real, >= 0
  const double den = sqrt(a.re * a.re + a.im * a.im + bb * bb);
  cplx c, sv;
  if (den > 0.0) {
    c = cplx{a.re / den, a.im / den};
    sv = cplx{bb / den, 0.0};
  } else {
    c = cplx{1.0, 0.0};
    sv = cplx{0.0, 0.0};
  }
  cs[k] = c;
  sn[k] = sv;
  Hc[k] = cplx{den, 0.0};
  Hc[k + 1] = cplx{0.0, 0.0};
  const cplx gk = g[k];
  g[k + 1] = cplx{-(sv.re * gk.re - sv.im * gk.im), -(sv.re * gk.im + sv.im * gk.re)};
  g[k] = cplx{c.re * gk.re + c.im * gk.im, c.re * gk.im - c.im * gk.re};
  const double r = sqrt(g[k + 1].re * g[k + 1].re + g[k + 1].im * g[k + 1].im);
  d.res[s] = r;
  d.norm[q] = nrm;
  const int knew = k + 1;
  d.kk[s] = knew;
  int f = 0;
  if (!(r == r) || !(nrm == nrm) || std::isinf(r)) f = 3;              // non-finite
  else if (r <= d.ctol[s] || knew >= m || nrm == 0.0 || iters_left_any == 0) f = 1;
  flags_out[q] = f;
  k_out[q] = knew;
  res_out[q] = r;
  if (f != 0) {
    d.flag[s] = f;
    d.fresh[s] = 1;
  }
}

// V[k] (new) *= 1/||w||  (k already advanced)
__global__ void scale_kernel(SolverDev d, const int* act) {
  const int q = blockIdx.y;
  const int s = act[q];
  if (d.flag[s] != 0 && d.fresh[s] == 0) return;
  const int k = d.kk[s];
  const double nrm = d.norm[q];
  const double f = nrm > 0.0 ? 1.0 / nrm : 0.0;
  double* vr = vec(d, s, k, 0);
  double* vi = vec(d, s, k, 1);
  const int64_t i0 = int64_t(blockIdx.x) * CH;
  for (int e = threadIdx.x; e < CH; e += VT) {
    const int64_t t = i0 + e;
    if (t < d.Dp) {
      vr[t] *= f;
      vi[t] *= f;
    }
  }
}

// drop the current cycle of the listed slots (k = 0: the solution update adds nothing)
__global__ void drop_cycle_kernel(SolverDev d, const int* slots, int n) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) d.kk[slots[q]] = 0;
}

// y = R^-1 g (upper triangular k x k) per finishing slot
__global__ void trisolve_kernel(SolverDev d, const int* fin, int n) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const int s = fin[q];
  const int k = d.kk[s];
  const int m = d.m;
  const cplx* H = d.H + int64_t(s) * m * (m + 1);
  const cplx* g = d.g + int64_t(s) * (m + 1);
  cplx* y = d.y + int64_t(s) * m;
  for (int i = k - 1; i >= 0; --i) {
    double ar = g[i].re, ai = g[i].im;
    for (int j = i + 1; j < k; ++j) {
      const cplx hij = H[int64_t(j) * (m + 1) + i];
      ar -= hij.re * y[j].re - hij.im * y[j].im;
      ai -= hij.re * y[j].im + hij.im * y[j].re;
    }
    const cplx hii = H[int64_t(i) * (m + 1) + i];
    const double den = hii.re * hii.re + hii.im * hii.im;
    if (den > 0.0)
      y[i] = cplx{(ar * hii.re + ai * hii.im) / den, (ai * hii.re - ar * hii.im) / den};
    else
      y[i] = cplx{0.0, 0.0};
  }
}

// X += M^-1 sum_j y_j V_j (or sum_j y_j Z_j), and copy X into the dense planes
__global__ void xupdate_kernel(SolverDev d, const int* fin, double* xout, const double* diag, int mode, int flex) {
  const int q = blockIdx.y;
  const int s = fin[q];
  const int k = d.kk[s];
  const cplx z = d.z[s];
  const cplx* y = d.y + int64_t(s) * d.m;
  double* xr = d.X + (int64_t(s) * 2) * d.Dp;
  double* xi = xr + d.Dp;
  const int64_t i0 = int64_t(blockIdx.x) * CH;
  for (int e = threadIdx.x; e < CH; e += VT) {
    const int64_t t = i0 + e;
    if (t >= d.Dp) break;
    double ar = 0.0, ai = 0.0;
    for (int j = 0; j < k; ++j) {
      const double* b = flex ? d.Z + ((int64_t(s) * d.m + j) * 2) * d.Dp : vec(d, s, j, 0);
      const double br = b[t], bi = b[d.Dp + t];
      ar += y[j].re * br - y[j].im * bi;
      ai += y[j].re * bi + y[j].im * br;
    }
    if (!flex && mode == GFCC_PC_JACOBI) {
      const double dr = z.re + diag[t], di = z.im;
      const double den = 1.0 / (dr * dr + di * di);
      const double nr = (ar * dr + ai * di) * den, ni = (ai * dr - ar * di) * den;
      ar = nr;
      ai = ni;
    }
    xr[t] += ar;
    xi[t] += ai;
    xout[(int64_t(q) * 2) * d.Dp + t] = xr[t];
    xout[(int64_t(q) * 2 + 1) * d.Dp + t] = xi[t];
  }
}

// r = b - z x - sigma(x) -> V[0]; partial ||r||^2 (b = e_p when brow < 0)
__global__ void residual_kernel(SolverDev d, const int* fin, const int* pfin, const int* brow, const double* brows,
                                const double* xin, const double* sig) {
  const int q = blockIdx.y;
  const int s = fin[q];
  const cplx z = d.z[s];
  const int p = pfin[q];
  const double* bp = brow[q] < 0 ? nullptr : brows + int64_t(brow[q]) * d.Dp;
  double* r0 = vec(d, s, 0, 0);
  double* r1 = vec(d, s, 0, 1);
  const double* xr = xin + (int64_t(q) * 2) * d.Dp;
  const double* sr = sig + (int64_t(q) * 2) * d.Dp;
  const int64_t i0 = int64_t(blockIdx.x) * CH;
  double acc = 0.0;
  for (int e = threadIdx.x; e < CH; e += VT) {
    const int64_t t = i0 + e;
    if (t >= d.Dp) break;
    const double a = xr[t], b = xr[d.Dp + t];
    double rr = -(z.re * a - z.im * b) - sr[t];
    const double ri = -(z.re * b + z.im * a) - sr[d.Dp + t];
    if (bp)
      rr += bp[t];
    else if (t == p)
      rr += 1.0;
    r0[t] = rr;
    r1[t] = ri;
    acc += rr * rr + ri * ri;
  }
  __shared__ double red[VT / 64];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int w = 0; w < VT / 64; ++w) t += red[w];
    d.npart[int64_t(q) * d.nch + blockIdx.x] = t;
  }
}

__global__ void rnorm_kernel(SolverDev d, int n, double* beta) {
  const int q = blockIdx.x;
  if (q >= n) return;
  __shared__ double red[64];
  double acc = 0.0;
  for (int c = threadIdx.x; c < d.nch; c += 64) acc += d.npart[int64_t(q) * d.nch + c];
  red[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int w = 0; w < 64; ++w) t += red[w];
    beta[q] = sqrt(t);
  }
}

// restart: V0 = r / beta, g = (beta, 0, ...), k = 0, new cycle tolerance
__global__ void restart_kernel(SolverDev d, const int* slots, const double* beta, const double* ctol, int n) {
  const int q = blockIdx.y;
  if (q >= n) return;
  const int s = slots[q];
  const double b = beta[q];
  const double f = b > 0.0 ? 1.0 / b : 0.0;
  double* r0 = vec(d, s, 0, 0);
  double* r1 = vec(d, s, 0, 1);
  const int64_t i0 = int64_t(blockIdx.x) * CH;
  for (int e = threadIdx.x; e < CH; e += VT) {
    const int64_t t = i0 + e;
    if (t < d.Dp) {
      r0[t] *= f;
      r1[t] *= f;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    d.kk[s] = 0;
    d.flag[s] = 0;
    d.fresh[s] = 0;
    d.ctol[s] = ctol[q];
    d.res[s] = b;
    for (int j = 0; j <= d.m; ++j) d.g[int64_t(s) * (d.m + 1) + j] = cplx{j == 0 ? b : 0.0, 0.0};
  }
}

// G[row][k] = c_{q_k} . x  for finished slots; the left vector is row
// qrow[k] of `left`, or row crow[f] (the slot's own p) when qrow is null
__global__ void gdot_kernel(SolverDev d, const int* slots, const int64_t* rows, const int* crow, const int64_t* qrow,
                            int nq, const double* left, double* G) {
  const int f = blockIdx.x;
  const int kq = blockIdx.y;
  const int s = slots[f];
  const int64_t qq = qrow ? qrow[kq] : crow[f];
  const double* c = left + qq * d.Dp;
  const double* xr = d.X + (int64_t(s) * 2) * d.Dp;
  const double* xi = xr + d.Dp;
  double a = 0.0, b = 0.0;
  for (int64_t t = threadIdx.x; t < d.Dp; t += VT) {
    a += c[t] * xr[t];
    b += c[t] * xi[t];
  }
  __shared__ double red[VT / 64][2];
  a = wave_sum(a);
  b = wave_sum(b);
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6][0] = a;
    red[threadIdx.x >> 6][1] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double ta = 0, tb = 0;
    for (int w = 0; w < VT / 64; ++w) {
      ta += red[w][0];
      tb += red[w][1];
    }
    G[(rows[f] * nq + kq) * 2] = ta;
    G[(rows[f] * nq + kq) * 2 + 1] = tb;
  }
}

// |row r| of rows [n][Dp]
__global__ void row_norm_kernel(const double* rows, int64_t Dp, double* out) {
  const int64_t r = blockIdx.x;
  double acc = 0.0;
  for (int64_t t = threadIdx.x; t < Dp; t += VT) {
    const double x = rows[r * Dp + t];
    acc += x * x;
  }
  __shared__ double red[VT / 64];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int w = 0; w < VT / 64; ++w) t += red[w];
    out[r] = sqrt(t);
  }
}

// copy X of finished slots to the caller's interleaved [nrhs][D] array
__global__ void xout_kernel(SolverDev d, const int* slots, const int64_t* rows, double* Xo, int64_t D, int64_t o,
                            int64_t o_pad) {
  const int f = blockIdx.y;
  const int s = slots[f];
  const double* xr = d.X + (int64_t(s) * 2) * d.Dp;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < D; t += int64_t(gridDim.x) * blockDim.x) {
    const int64_t src = t < o ? t : t - o + o_pad;
    Xo[(rows[f] * D + t) * 2] = xr[src];
    Xo[(rows[f] * D + t) * 2 + 1] = xr[d.Dp + src];
  }
}

// ------------------------------------------------------------------ host driver

struct HostSlot {
  int64_t rhs = -1;
  int iters = 0, restarts = 0;
  int k = 0;               // Krylov step (mirror of the device counter)
  int mlp = 0;             // 1 while the learned preconditioner is in use
  bool fell_back = false;  // switched to Jacobi after an MLP cycle stalled
  bool nonfinite = false;  // the current cycle produced a non-finite value
  double beta = 1.0;       // residual at the start of the current cycle
  double bn = 1.0;         // |b_p|
  int brow = -1;           // row of b_p in the materialised right-hand sides (-1: e_p)
  double ctol = 0.0;       // the current cycle's target for the residual estimate
  double res = 1.0;        // residual estimate at the last synchronisation
  double lrate = 0.0;      // log of its reduction per iteration (0: not observed yet)
};

// Page-locked host memory: device-to-host copies into it stay asynchronous.
struct HBuf {
  void* p = nullptr;
  size_t bytes = 0;
  HBuf() = default;
  HBuf(const HBuf&) = delete;
  HBuf& operator=(const HBuf&) = delete;
  HBuf(HBuf&& o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
  HBuf& operator=(HBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; bytes = o.bytes; o.p = nullptr; o.bytes = 0; }
    return *this;
  }
  ~HBuf() { release(); }
  void release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
  }
  void ensure(size_t n) {
    if (n <= bytes && p) return;
    release();
    if (hipHostMalloc(&p, n, hipHostMallocDefault) != hipSuccess) {
      p = nullptr;
      throw Error{GFCC_E_OOM, "hipHostMalloc of " + std::to_string(n) + " bytes failed"};
    }
    bytes = n;
  }
  template <typename T> T* as() const { return static_cast<T*>(p); }
};

static double lp_cycle_rtol(gfcc_precision p) {
  switch (p) {
    case GFCC_FP32_IR: return 1e-6;
    case GFCC_BF16_IR: return 1e-4;
    case GFCC_FP16_IR: return 2e-5;  // three more mantissa bits than BF16
    default: return 0.0;
  }
}

// One system's share of the solve: a window of B slots on its context, the
// queue of its right-hand sides (global indices) and the device state.
struct Lane {
  gfcc_ctx* c = nullptr;
  std::vector<int64_t> rows;
  size_t next = 0;
  int B = 0, nch = 0;
  int defer = 0;  // inner iterations cycle finishing has waited for the last active slots
  int64_t Dp = 0;
  DBuf bV, bZ, bX, bH, bcs, bsn, bg, by, bz, bkk, bctol, bres, bflag, bfresh, bpart, bGm, bh, bnpart, bnorm;
  SolverDev d{};
  DBuf d_act, d_stat, d_list, d_plist, d_brow, d_zlist, d_ctl, d_beta, d_rows, d_q;
  DBuf d_msrc, d_mzoff, d_mom, d_pmode;
  DBuf d_ag, d_agb, d_agt, d_drop;  // restart and dropped-cycle lists of cycle finishing
  std::map<int64_t, int> brow_of;  // virtual p -> row of bB
  std::vector<double> bnorm_h;
  DBuf d_borb, bB, bBn;
  const double* lrows = nullptr;
  std::map<int64_t, int64_t> lrow_of;
  DBuf d_lorb, bL;
  std::vector<HostSlot> hs;
  std::vector<int> free_slots, active, pending;
  std::vector<int> act_dev;  // the active list as last uploaded to d_act
  HBuf hstat;                // page-locked copy of d_stat
  std::vector<double> hbeta;
  int64_t lrow(int64_t orb) const { return lrow_of.empty() ? orb : lrow_of.at(orb); }
};

namespace {

struct BatchRun {
  const int64_t* p;
  const double* omega;
  double eta;
  int64_t nq;
  const int64_t* q;
  const gfcc_solve_opts* opts;
  double* G;
  double* Xout;
  gfcc_rhs_info* info;
  PairRec* rec;
  hipStream_t s;
  int m = 0, mode = 0, flex = 0;
  bool use_mlp = false;
  gfcc_precision prec = GFCC_FP64;
  double tol = 0.0, rtol_lp = 0.0;
  bool ok_all = true;
  int64_t n_sync = 0;        // host synchronisations of the run
  int64_t n_loop_sync = 0;   // of which after inner iterations
  int64_t n_iter = 0;        // inner iterations launched (one per window step)
  int64_t n_plane_iter = 0;  // right-hand-side iterations launched (frozen slots included)

  void sync(hipStream_t st) {
    ++n_sync;
    GFCC_HIP(hipStreamSynchronize(st));
    stage_off = 0;  // every staged copy has completed
  }

  // Host-to-device copies of small lists go through page-locked staging memory,
  // so they are asynchronous and need no synchronisation before the host list
  // goes away; the staging area is reused after the next synchronisation.
  HBuf stage;
  size_t stage_off = 0;
  template <typename T>
  void upload(DBuf& b, const std::vector<T>& v, hipStream_t st) {
    b.ensure(std::max<size_t>(v.size(), 1) * sizeof(T), st);
    if (v.empty()) return;
    const size_t n = v.size() * sizeof(T);
    size_t off = (stage_off + 15) & ~size_t(15);
    if (off + n > stage.bytes) {
      if (stage_off > 0) sync(st);
      stage.ensure(std::max(n, size_t(1) << 20));
      off = 0;
    }
    std::memcpy(stage.as<char>() + off, v.data(), n);
    GFCC_HIP(hipMemcpyAsync(b.p, stage.as<char>() + off, n, hipMemcpyHostToDevice, st));
    stage_off = off + n;
  }

  // Resume file: a header (magic, version, record size, fingerprint of the
  // request), then one record per finished right-hand side, appended as it finishes.
  struct CkptHeader {
    char magic[8];
    int32_t version, rec_size;
    uint64_t fingerprint;
  };
  struct CkptRec {
    int64_t row, p, nq, qhash;
    double omega, eta;
    gfcc_rhs_info info;
  };  // followed by 2 nq doubles (the G row)
  static constexpr char kMagic[8] = {'G', 'F', 'C', 'C', 'R', 'E', 'S', 'M'};
  static constexpr int32_t kVersion = 2;
  FILE* ck = nullptr;
  std::set<int64_t> restored;
  int64_t qhash = 0;
  const int32_t* sysv = nullptr;  // system of each right-hand side (several-system solves)

  // FNV-1a over the request: every system's dimensions and a sample of its exact
  // diagonal, the system of each right-hand side, the q list, eta and the solver
  // options that change results (tolerance, precision, preconditioner, restart,
  // max_iter).  p and omega are matched per record.
  uint64_t fingerprint(const std::vector<Lane>& lanes, int64_t nrhs) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](uint64_t x) {
      for (int b = 0; b < 8; ++b) {
        h ^= (x >> (8 * b)) & 0xffu;
        h *= 1099511628211ull;
      }
    };
    auto mixd = [&](double x) {
      uint64_t u;
      std::memcpy(&u, &x, 8);
      mix(u);
    };
    mix(uint64_t(lanes.size()));
    for (const Lane& L : lanes) {
      const gfcc_ctx* c = L.c;
      mix(uint64_t(c->o));
      mix(uint64_t(c->v));
      mix(uint64_t(c->sector));
      mix(uint64_t(c->Q));
      const int64_t n = std::min<int64_t>(c->Dp, 2048);
      std::vector<double> dg(size_t(2 * n));
      GFCC_HIP(hipMemcpyAsync(dg.data(), c->diag.p, size_t(n) * 8, hipMemcpyDeviceToHost, s));
      GFCC_HIP(hipMemcpyAsync(dg.data() + n, c->diag.as<double>() + (c->Dp - n), size_t(n) * 8,
                              hipMemcpyDeviceToHost, s));
      sync(s);
      for (double x : dg) mixd(x);
    }
    if (sysv)
      for (int64_t r = 0; r < nrhs; ++r) mix(uint64_t(sysv[r]));
    mix(uint64_t(nq));
    for (int64_t k = 0; q && k < nq; ++k) mix(uint64_t(q[k]));
    mixd(eta);
    mixd(opts->tol);
    mix(uint64_t(opts->precision));
    mix(uint64_t(opts->precond));
    mix(uint64_t(opts->restart));
    mix(uint64_t(opts->max_iter));
    return h;
  }

  // Restore the rows a previous call recorded for this request, then open the file
  // for appending.  A file that is not a resume file, or belongs to another request,
  // is refused with E_ARG and left untouched.
  void ckpt_open(const std::vector<Lane>& lanes, int64_t nrhs) {
    if (!opts->checkpoint) return;
    uint64_t h = 1469598103934665603ull;  // FNV-1a over (nq, q): matched per record
    auto mix = [&](int64_t x) {
      for (int b = 0; b < 8; ++b) {
        h ^= uint64_t(x >> (8 * b)) & 0xffu;
        h *= 1099511628211ull;
      }
    };
    mix(nq);
    for (int64_t k = 0; q && k < nq; ++k) mix(q[k]);
    if (!q) mix(-1);
    qhash = int64_t(h);
    CkptHeader want{};
    std::memcpy(want.magic, kMagic, 8);
    want.version = kVersion;
    want.rec_size = int32_t(sizeof(CkptRec));
    want.fingerprint = fingerprint(lanes, nrhs);
    std::vector<double> gbuf;
    std::vector<int64_t> rows;
    long good = 0, total = 0;  // bytes of the header and whole records / of the file
    bool fresh = true;
    if (FILE* f = std::fopen(opts->checkpoint, "rb")) {
      std::fseek(f, 0, SEEK_END);
      total = std::ftell(f);
      std::fseek(f, 0, SEEK_SET);
      if (total > 0) {
        fresh = false;
        CkptHeader got{};
        const bool hdr = std::fread(&got, sizeof(got), 1, f) == 1 && std::memcmp(got.magic, kMagic, 8) == 0 &&
                         got.version == kVersion && got.rec_size == int32_t(sizeof(CkptRec));
        if (!hdr) {
          std::fclose(f);
          throw Error{GFCC_E_ARG, std::string("not a resume file of this library: ") + opts->checkpoint};
        }
        if (got.fingerprint != want.fingerprint) {
          std::fclose(f);
          throw Error{GFCC_E_ARG, std::string("resume file belongs to a different request (system, q, eta or "
                                              "solver options): ") + opts->checkpoint};
        }
        good = long(sizeof(CkptHeader));
        CkptRec r;
        std::vector<double> g;
        while (std::fread(&r, sizeof(r), 1, f) == 1) {
          if (r.nq < 1 || r.nq > (int64_t(1) << 20)) break;  // torn or corrupt tail
          g.resize(size_t(2 * r.nq));
          if (std::fread(g.data(), sizeof(double), g.size(), f) != g.size()) break;
          good = std::ftell(f);
          if (r.nq != nq) continue;
          const bool same = r.row >= 0 && r.row < nrhs && r.p == p[r.row] && r.omega == omega[r.row] &&
                            r.eta == eta && r.qhash == qhash;
          if (!same || restored.count(r.row)) continue;
          restored.insert(r.row);
          info[r.row] = r.info;
          if (r.info.status != 0 && r.info.status != 4) ok_all = false;
          rows.push_back(r.row);
          gbuf.insert(gbuf.end(), g.begin(), g.end());
        }
      }
      std::fclose(f);
    }
    // a record torn by an interrupted write is cut off (after a valid header) before appending
    if (!fresh && total > good)
      GFCC_CHECK(::truncate(opts->checkpoint, good) == 0, GFCC_E_ARG, "cannot trim resume file");
    for (size_t k = 0; k < rows.size(); ++k) {
      GFCC_HIP(hipMemcpyAsync(G + rows[k] * nq * 2, gbuf.data() + k * 2 * nq, size_t(nq) * 16,
                              hipMemcpyHostToDevice, s));
      if (Xout) {  // restored rows carry no solution
        const int64_t D = lanes[0].c->D;
        GFCC_HIP(hipMemsetAsync(Xout + rows[k] * D * 2, 0, size_t(D) * 16, s));
      }
    }
    sync(s);  // gbuf goes out of scope
    ck = std::fopen(opts->checkpoint, fresh ? "wb" : "ab");
    GFCC_CHECK(ck, GFCC_E_ARG, std::string("cannot open resume file ") + opts->checkpoint);
    if (fresh) {
      std::fwrite(&want, sizeof(want), 1, ck);
      std::fflush(ck);
    }
  }

  // append the finished rows (G already on the device)
  void ckpt_write(const std::vector<int64_t>& rows) {
    if (!ck || rows.empty()) return;
    std::vector<double> g(rows.size() * size_t(2 * nq));
    for (size_t k = 0; k < rows.size(); ++k)
      GFCC_HIP(hipMemcpyAsync(g.data() + k * 2 * nq, G + rows[k] * nq * 2, size_t(nq) * 16,
                              hipMemcpyDeviceToHost, s));
    sync(s);
    for (size_t k = 0; k < rows.size(); ++k) {
      const int64_t r = rows[k];
      CkptRec rec{r, p[r], nq, qhash, omega[r], eta, info[r]};
      std::fwrite(&rec, sizeof(rec), 1, ck);
      std::fwrite(g.data() + k * 2 * nq, sizeof(double), size_t(2 * nq), ck);
    }
    std::fflush(ck);
  }

  void ckpt_close() {
    if (ck) std::fclose(ck);
    ck = nullptr;
  }

  // device buffers, right-hand-side rows and left rows of one lane
  void setup(Lane& L) {
    gfcc_ctx* c = L.c;
    const int B = L.B;
    const int64_t Dp = c->Dp;
    L.Dp = Dp;
    L.nch = int((Dp + CH - 1) / CH);
    const int nch = L.nch;
    L.bV.ensure(size_t(B) * (m + 1) * 2 * Dp * 8, s);
    if (flex) L.bZ.ensure(size_t(B) * m * 2 * Dp * 8, s);
    L.bX.ensure(size_t(B) * 2 * Dp * 8, s);
    L.bH.ensure(size_t(B) * m * (m + 1) * sizeof(cplx), s);
    L.bcs.ensure(size_t(B) * m * sizeof(cplx), s);
    L.bsn.ensure(size_t(B) * m * sizeof(cplx), s);
    L.bg.ensure(size_t(B) * (m + 1) * sizeof(cplx), s);
    L.by.ensure(size_t(B) * m * sizeof(cplx), s);
    L.bz.ensure(size_t(B) * sizeof(cplx), s);
    L.bkk.ensure(size_t(B) * sizeof(int), s);
    L.bctol.ensure(size_t(B) * 8, s);
    L.bres.ensure(size_t(B) * 8, s);
    L.bflag.ensure(size_t(B) * sizeof(int), s);
    L.bfresh.ensure(size_t(B) * sizeof(int), s);
    L.bpart.ensure(size_t(B) * nch * PS * sizeof(cplx), s);
    L.bGm.ensure(size_t(B) * m * (m + 1) * sizeof(cplx), s);
    L.bh.ensure(size_t(B) * (MAXM + 1) * sizeof(cplx), s);
    L.bnpart.ensure(size_t(B) * nch * 8, s);
    L.bnorm.ensure(size_t(B) * 8, s);
    c->ws_in.ensure(size_t(2 * B) * Dp * 8, s);
    c->ws_out.ensure(size_t(2 * B) * Dp * 8, s);
    SolverDev& d = L.d;
    d.V = L.bV.as<double>();
    d.Z = flex ? L.bZ.as<double>() : nullptr;
    d.X = L.bX.as<double>();
    d.H = L.bH.as<cplx>();
    d.cs = L.bcs.as<cplx>();
    d.sn = L.bsn.as<cplx>();
    d.g = L.bg.as<cplx>();
    d.y = L.by.as<cplx>();
    d.z = L.bz.as<cplx>();
    d.kk = L.bkk.as<int>();
    d.ctol = L.bctol.as<double>();
    d.res = L.bres.as<double>();
    d.flag = L.bflag.as<int>();
    d.fresh = L.bfresh.as<int>();
    d.part = L.bpart.as<cplx>();
    d.Gm = L.bGm.as<cplx>();
    d.h = L.bh.as<cplx>();
    d.npart = L.bnpart.as<double>();
    d.norm = L.bnorm.as<double>();
    d.m = m;
    d.Dp = Dp;
    d.nch = nch;
    L.d_stat.ensure(size_t(B) * 16, s);  // flags, Krylov steps, residual estimates
    L.hstat.ensure(size_t(B) * 16);
    L.d_beta.ensure(size_t(B) * 8, s);
    // lists of at most B entries, sized once so that cycle finishing allocates nothing
    for (DBuf* b : {&L.d_act, &L.d_list, &L.d_plist, &L.d_brow, &L.d_ag, &L.d_agt, &L.d_drop})
      b->ensure(size_t(B) * 8, s);
    for (DBuf* b : {&L.d_zlist, &L.d_ctl, &L.d_agb, &L.d_rows}) b->ensure(size_t(B) * 16, s);

    // Right-hand sides of virtual orbitals, one materialised row per distinct
    // orbital with its norm; occupied p keep the implicit unit vector e_p.
    std::vector<int64_t> borb;
    for (int64_t r : L.rows)
      if (c->materialised(p[r]) && !L.brow_of.count(p[r])) {
        L.brow_of[p[r]] = int(borb.size());
        borb.push_back(p[r]);
      }
    L.bnorm_h.assign(borb.size(), 0.0);
    if (!borb.empty()) {
      const int64_t nb = int64_t(borb.size());
      upload(L.d_borb, borb, s);
      L.bB.ensure(size_t(nb * Dp) * 8, s);
      L.bBn.ensure(size_t(nb) * 8, s);
      make_rhs_rows(c, nb, L.d_borb.as<int64_t>(), L.bB.as<double>(), s);
      hipLaunchKernelGGL(row_norm_kernel, dim3(unsigned(nb)), dim3(VT), 0, s, L.bB.as<double>(), Dp,
                         L.bBn.as<double>());
      GFCC_HIP(hipGetLastError());
      GFCC_HIP(hipMemcpyAsync(L.bnorm_h.data(), L.bBn.p, size_t(nb) * 8, hipMemcpyDeviceToHost, s));
      sync(s);
    }
    // Left vectors: the occupied rows built with the intermediates, or, when a
    // virtual orbital is asked for, one materialised row per distinct orbital.
    L.lrows = c->left.as<double>();
    bool virt = false;
    if (q) {
      for (int64_t k = 0; k < nq; ++k) virt = virt || c->materialised(q[k]);
    } else {
      virt = !borb.empty();
    }
    if (virt) {
      std::vector<int64_t> lorb;
      auto add = [&](int64_t orb) {
        if (!L.lrow_of.count(orb)) {
          L.lrow_of[orb] = int64_t(lorb.size());
          lorb.push_back(orb);
        }
      };
      if (q)
        for (int64_t k = 0; k < nq; ++k) add(q[k]);
      else
        for (int64_t r : L.rows) add(p[r]);
      upload(L.d_lorb, lorb, s);
      L.bL.ensure(lorb.size() * size_t(Dp) * 8, s);
      make_left_rows(c, int64_t(lorb.size()), L.d_lorb.as<int64_t>(), L.bL.as<double>(), s);
      L.lrows = L.bL.as<double>();
    }
    if (q) {
      std::vector<int64_t> qr(static_cast<size_t>(nq));
      for (int64_t k = 0; k < nq; ++k) qr[size_t(k)] = L.lrow(q[k]);
      upload(L.d_q, qr, s);
    }
    L.hs.assign(size_t(B), HostSlot{});
    for (int i = B - 1; i >= 0; --i) L.free_slots.push_back(i);
    L.hbeta.assign(size_t(B), 0.0);
    sync(s);
  }

  void refill(Lane& L) {
    gfcc_ctx* c = L.c;
    std::vector<int> sl, pl, bl;
    std::vector<cplx> zl;
    std::vector<double> tl;
    std::vector<int64_t> zero_rows;
    while (!L.free_slots.empty() && L.next < L.rows.size()) {
      const int64_t r = L.rows[L.next];
      if (restored.count(r)) {  // finished in an earlier call (resume file)
        ++L.next;
        continue;
      }
      const int br = c->materialised(p[r]) ? L.brow_of.at(p[r]) : -1;
      const double bn = br < 0 ? 1.0 : L.bnorm_h[size_t(br)];
      if (!(bn > 0.0)) {  // b_p = 0 (no amplitude reaches this orbital): X = 0, G = 0
        info[r] = gfcc_rhs_info{0, 0, 0, 0, 0.0};
        GFCC_HIP(hipMemsetAsync(G + r * nq * 2, 0, size_t(nq) * 16, s));
        if (Xout) GFCC_HIP(hipMemsetAsync(Xout + r * c->D * 2, 0, size_t(c->D) * 16, s));
        zero_rows.push_back(r);
        ++L.next;
        continue;
      }
      const int sidx = L.free_slots.back();
      L.free_slots.pop_back();
      HostSlot& h = L.hs[size_t(sidx)];
      h = HostSlot{};
      h.rhs = r;
      h.mlp = use_mlp ? 1 : 0;
      h.bn = bn;
      h.beta = bn;
      h.brow = br;
      h.res = bn;
      h.ctol = bn * std::max(0.5 * tol, rtol_lp);
      sl.push_back(sidx);
      pl.push_back(int(p[r]));
      bl.push_back(br);
      zl.push_back(cplx{omega[r], -eta});
      tl.push_back(h.ctol);
      L.active.push_back(sidx);
      ++L.next;
    }
    ckpt_write(zero_rows);
    if (sl.empty()) return;
    upload(L.d_list, sl, s);
    upload(L.d_plist, pl, s);
    upload(L.d_brow, bl, s);
    upload(L.d_zlist, zl, s);
    upload(L.d_ctl, tl, s);
    hipLaunchKernelGGL(init_slots_kernel, dim3(L.nch, unsigned(sl.size())), dim3(VT), 0, s, L.d, L.d_list.as<int>(),
                       L.d_plist.as<int>(), L.d_brow.as<int>(), L.bB.as<double>(), L.bBn.as<double>(),
                       L.d_zlist.as<cplx>(), L.d_ctl.as<double>(), int(sl.size()));
    GFCC_HIP(hipGetLastError());
  }

  // preconditioner step of one inner iteration: u = M^-1 V[k] into ws_in
  void pre(Lane& L, hipStream_t st) {
    gfcc_ctx* c = L.c;
    const int na = int(L.active.size());
    const int* act = L.d_act.as<int>();
    SolverDev& d = L.d;
    if (!use_mlp) {
      hipLaunchKernelGGL(precond_kernel, dim3(L.nch, na), dim3(VT), 0, st, d, act, c->ws_in.as<double>(),
                         c->diag.as<double>(), mode, flex);
      GFCC_HIP(hipGetLastError());
      return;
    }
    std::vector<int> sidx(na), pm(L.B);
    std::vector<int64_t> zoff(na);
    std::vector<double> om(na);
    for (int i = 0; i < na; ++i) {
      const int sl = L.active[size_t(i)];
      sidx[i] = sl * (m + 1) + L.hs[size_t(sl)].k;
      zoff[i] = ((int64_t(sl) * m + L.hs[size_t(sl)].k) * 2) * L.Dp;
      om[i] = omega[L.hs[size_t(sl)].rhs];
    }
    for (int sl = 0; sl < L.B; ++sl) pm[sl] = L.hs[size_t(sl)].mlp;
    upload(L.d_msrc, sidx, st);
    upload(L.d_mzoff, zoff, st);
    upload(L.d_mom, om, st);
    upload(L.d_pmode, pm, st);
    MlpApplyArgs a;
    a.src = d.V;
    a.src_idx = L.d_msrc.as<int>();
    a.slots = act;
    a.mode = L.d_pmode.as<int>();
    a.omega = L.d_mom.as<double>();
    a.nrm = nullptr;
    a.nrm_const = 1.0 / std::sqrt(double(c->D));  // Krylov vectors have unit norm
    a.eta = eta;
    a.dst = c->ws_in.as<double>();
    a.zdst = d.Z;
    a.zoff = L.d_mzoff.as<int64_t>();
    prof_begin(c, "mlp", st);
    mlp_apply(c, a, na, st);
    prof_end(c, "mlp", st, 2.0 * double(na) * double(c->D) *
                               (double(MLP_F) * c->mlp->width + double(c->mlp->width) * c->mlp->width +
                                2.0 * c->mlp->width), 0.0);
  }

  // CGS2 Arnoldi step and Givens update after the sigma
  void post(Lane& L, hipStream_t st) {
    gfcc_ctx* c = L.c;
    const int na = int(L.active.size());
    const int* act = L.d_act.as<int>();
    SolverDev& d = L.d;
    prof_begin(c, "arnoldi", st);
    hipLaunchKernelGGL(arnoldi_kernel, dim3(L.nch, na), dim3(VT), 0, st, d, act, c->ws_in.as<double>(),
                       c->ws_out.as<double>(), 0);
    hipLaunchKernelGGL(reduce_hg_kernel, dim3(na), dim3(MAXM + 1), 0, st, d, act);
    hipLaunchKernelGGL(arnoldi_kernel, dim3(L.nch, na), dim3(VT), 0, st, d, act, c->ws_in.as<double>(),
                       c->ws_out.as<double>(), 2);
    GFCC_HIP(hipGetLastError());
    hipLaunchKernelGGL(givens_kernel, dim3(na), dim3(64), 0, st, d, act, L.d_stat.as<int>(), L.B, 1);
    hipLaunchKernelGGL(scale_kernel, dim3(L.nch, na), dim3(VT), 0, st, d, act);
    GFCC_HIP(hipGetLastError());
    if (c->prof_on) {
      // algorithmic HBM bytes of the step, per slot at Krylov step k (planes of Dp doubles):
      // pass 0 reads u, sigma and V_k (6) and the k+1 basis vectors (2(k+1)), writes w (2);
      // pass 2 reads the basis again (2(k+1)) and w (2), writes w (2); the scaling reads and
      // writes w (4)
      double planes = 0.0;
      for (int sl : L.active) planes += 4.0 * double(L.hs[size_t(sl)].k + 1) + 16.0;
      prof_end(c, "arnoldi", st, 0.0, planes * double(L.Dp) * 8.0);
    } else {
      prof_end(c, "arnoldi", st, 0.0, 0.0);
    }
  }

  // one inner iteration of every lane with active slots
  void iteration(std::vector<Lane*>& live, hipStream_t st) {
    for (Lane* L : live) pre(*L, st);
    if (live.size() == 1) {
      Lane& L = *live[0];
      sigma_planes(L.c, 2 * int64_t(L.active.size()), L.c->ws_in.as<double>(), L.c->ws_out.as<double>(), prec, st);
    } else {
      std::vector<SigmaJob> jobs;
      for (Lane* L : live)
        jobs.push_back(SigmaJob{L->c, 2 * int64_t(L->active.size()), L->c->ws_in.as<double>(),
                                L->c->ws_out.as<double>()});
      sigma_group(jobs.data(), int(jobs.size()), prec, st);
    }
    for (Lane* L : live) post(*L, st);
  }

  // finish the cycles of the pending slots of one lane (true residual, restart or G)
  void finish(Lane& L) {
    gfcc_ctx* c = L.c;
    SolverDev& d = L.d;
    const int64_t Dp = L.Dp;
    std::vector<int> fin;
    fin.swap(L.pending);
    const int nf = int(fin.size());
    std::vector<int> pf(nf), bf(nf);
    for (int i = 0; i < nf; ++i) {
      pf[i] = int(p[L.hs[size_t(fin[i])].rhs]);
      bf[i] = L.hs[size_t(fin[i])].brow;
    }
    upload(L.d_list, fin, s);
    upload(L.d_plist, pf, s);
    upload(L.d_brow, bf, s);
    const int* fl = L.d_list.as<int>();
    // A cycle of the learned preconditioner that went non-finite (e.g. non-finite
    // network weights) is discarded: X keeps its value from before the cycle, the
    // true residual below then shows no progress and Jacobi takes over.
    std::vector<int> dropped;
    for (int i = 0; i < nf; ++i) {
      HostSlot& h = L.hs[size_t(fin[i])];
      if (h.nonfinite && h.mlp) dropped.push_back(fin[i]);
    }
    if (!dropped.empty()) {
      upload(L.d_drop, dropped, s);
      hipLaunchKernelGGL(drop_cycle_kernel, dim3((unsigned(dropped.size()) + 63) / 64), dim3(64), 0, s, d,
                         L.d_drop.as<int>(), int(dropped.size()));
      GFCC_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(trisolve_kernel, dim3((nf + 63) / 64), dim3(64), 0, s, d, fl, nf);
    hipLaunchKernelGGL(xupdate_kernel, dim3(L.nch, nf), dim3(VT), 0, s, d, fl, c->ws_in.as<double>(),
                       c->diag.as<double>(), mode, flex);
    GFCC_HIP(hipGetLastError());
    sigma_planes(c, 2 * nf, c->ws_in.as<double>(), c->ws_out.as<double>(), GFCC_FP64, s);
    hipLaunchKernelGGL(residual_kernel, dim3(L.nch, nf), dim3(VT), 0, s, d, fl, L.d_plist.as<int>(),
                       L.d_brow.as<int>(), L.bB.as<double>(), c->ws_in.as<double>(), c->ws_out.as<double>());
    hipLaunchKernelGGL(rnorm_kernel, dim3(nf), dim3(64), 0, s, d, nf, L.d_beta.as<double>());
    GFCC_HIP(hipGetLastError());
    GFCC_HIP(hipMemcpyAsync(L.hbeta.data(), L.d_beta.p, nf * 8, hipMemcpyDeviceToHost, s));
    sync(s);

    std::vector<int> done, again, done_p;
    std::vector<int64_t> done_rows;
    std::vector<double> again_beta, again_tol;
    for (int i = 0; i < nf; ++i) {
      const int sl = fin[i];
      HostSlot& h = L.hs[size_t(sl)];
      const double beta = L.hbeta[size_t(i)];  // |r|
      const double rel = beta / h.bn;
      const bool dropped_cycle = h.nonfinite && h.mlp;
      h.nonfinite = false;
      const bool finite = std::isfinite(beta);
      gfcc_rhs_info& inf = info[h.rhs];
      inf.iters = h.iters;
      inf.restarts = h.restarts;
      inf.true_rel_resid = rel;
      if (finite && rel <= tol) {
        inf.status = h.fell_back ? 4 : 0;
        if (rec) {  // keep X* of this right-hand side for the training pairs
          GFCC_HIP(hipMemcpyAsync(rec->xstar + h.rhs * 2 * Dp, d.X + int64_t(sl) * 2 * Dp, size_t(2 * Dp) * 8,
                                  hipMemcpyDeviceToDevice, s));
        }
      } else if (!finite) {
        inf.status = 3;
      } else if (h.iters >= opts->max_iter) {
        inf.status = 1;
        if (rec) {  // the last iterate, for pairs whose residual it undercuts by a wide margin
          GFCC_HIP(hipMemcpyAsync(rec->xstar + h.rhs * 2 * Dp, d.X + int64_t(sl) * 2 * Dp, size_t(2 * Dp) * 8,
                                  hipMemcpyDeviceToDevice, s));
          if (rec->final_nrm.size() <= size_t(h.rhs)) rec->final_nrm.resize(size_t(h.rhs) + 1, 0.0);
          rec->final_nrm[size_t(h.rhs)] = beta / std::sqrt(double(c->D));
        }
      } else {
        if (rec && rec->n < rec->cap) {  // (r_k, x_k) pair: V[s][0] holds the unnormalised residual
          GFCC_HIP(hipMemcpyAsync(rec->R + rec->n * 2 * Dp, d.V + int64_t(sl) * (m + 1) * 2 * Dp,
                                  size_t(2 * Dp) * 8, hipMemcpyDeviceToDevice, s));
          GFCC_HIP(hipMemcpyAsync(rec->X + rec->n * 2 * Dp, d.X + int64_t(sl) * 2 * Dp, size_t(2 * Dp) * 8,
                                  hipMemcpyDeviceToDevice, s));
          rec->rhs.push_back(int(h.rhs));
          rec->omega.push_back(omega[h.rhs]);
          rec->nrm.push_back(beta / std::sqrt(double(c->D)));
          rec->n += 1;
        }
        // the learned preconditioner hands over to Jacobi when a cycle stalls: it cut the true
        // residual by less than 10%, or it used the whole restart length without reaching
        // its cycle target
        if (h.mlp && (dropped_cycle || !(beta < 0.9 * h.beta) || h.k >= m)) {
          h.mlp = 0;
          h.fell_back = true;
        }
        h.beta = beta;
        h.k = 0;
        h.restarts += 1;
        h.res = beta;
        h.ctol = std::max(0.5 * tol * h.bn, rtol_lp * beta);
        again.push_back(sl);
        again_beta.push_back(beta);
        again_tol.push_back(h.ctol);
        continue;
      }
      if (inf.status != 0 && inf.status != 4) ok_all = false;
      done.push_back(sl);
      done_rows.push_back(h.rhs);
      done_p.push_back(q ? 0 : int(L.lrow(p[h.rhs])));  // own left vector only when q == NULL
    }
    if (!again.empty()) {
      const int nr = int(again.size());
      upload(L.d_ag, again, s);
      upload(L.d_agb, again_beta, s);
      upload(L.d_agt, again_tol, s);
      hipLaunchKernelGGL(restart_kernel, dim3(L.nch, nr), dim3(VT), 0, s, d, L.d_ag.as<int>(), L.d_agb.as<double>(),
                         L.d_agt.as<double>(), nr);
      GFCC_HIP(hipGetLastError());
    }
    if (!done.empty()) {
      const int nd = int(done.size());
      upload(L.d_list, done, s);
      upload(L.d_rows, done_rows, s);
      upload(L.d_plist, done_p, s);
      hipLaunchKernelGGL(gdot_kernel, dim3(nd, unsigned(nq)), dim3(VT), 0, s, d, L.d_list.as<int>(),
                         L.d_rows.as<int64_t>(), L.d_plist.as<int>(), q ? L.d_q.as<int64_t>() : nullptr, int(nq),
                         L.lrows, G);
      if (Xout)
        hipLaunchKernelGGL(xout_kernel, dim3(std::min<int64_t>((c->D + 255) / 256, 1024), nd), dim3(256), 0, s, d,
                           L.d_list.as<int>(), L.d_rows.as<int64_t>(), Xout, c->D, c->n1, c->p1);
      GFCC_HIP(hipGetLastError());
      ckpt_write(done_rows);  // copies the rows back and synchronises only with a resume file
      for (int sl : done) {
        L.hs[size_t(sl)].rhs = -1;
        L.free_slots.push_back(sl);
      }
    }
    for (int sl : again) L.active.push_back(sl);
    refill(L);
  }

  void run(std::vector<Lane>& lanes, int64_t nrhs) {
    struct Closer {
      BatchRun* r;
      ~Closer() { r->ckpt_close(); }
    } closer{this};
    ckpt_open(lanes, nrhs);
    for (auto& L : lanes) setup(L);
    if (opts->tune_cache) {  // ring-GEMM tiles for each full window (inner precision and FP64)
      const Prec ip = inner_prec(prec);
      for (auto& L : lanes) {
        if (L.c->sector != 0) continue;  // the tuned shapes are the ionisation sector's
        tune_load(L.c, opts->tune_cache);
        tune_ring(L.c, ip, 2 * int64_t(L.B), s);
        if (ip != Prec::F64) tune_ring(L.c, Prec::F64, 2 * int64_t(L.B), s);
        tune_save(L.c, opts->tune_cache);
      }
    }
    for (auto& L : lanes) refill(L);
    const bool any_prof = std::any_of(lanes.begin(), lanes.end(), [](const Lane& L) { return L.c->prof_on; });
    const bool graphable = opts->use_graph && !use_mlp && !any_prof;
    std::map<std::string, hipGraphExec_t> graphs;
    std::set<std::string> seen;
    struct GraphGuard {
      std::map<std::string, hipGraphExec_t>& g;
      ~GraphGuard() {
        for (auto& kv : g) (void)hipGraphExecDestroy(kv.second);
      }
    } graph_guard{graphs};
    struct CaptureStream {
      hipStream_t s = nullptr;
      ~CaptureStream() {
        if (s) (void)hipStreamDestroy(s);
      }
    } cap;
    uint64_t graph_gen = alloc_generation();
    for (;;) {
      std::vector<Lane*> live;
      bool work = false;
      for (auto& L : lanes) {
        if (!L.active.empty()) live.push_back(&L);
        work = work || !L.active.empty() || !L.pending.empty();
      }
      if (!work) break;
      if (!live.empty()) {
        std::string key;
        for (Lane* L : live) {
          if (L->act_dev != L->active) {  // the list on the device changes only with the active set
            upload(L->d_act, L->active, s);
            L->act_dev = L->active;
          }
          key += std::to_string(L->active.size()) + "@" + std::to_string(reinterpret_cast<uintptr_t>(L->d_act.p)) +
                 ";";
        }
        const int nb = burst(live);
        // One inner iteration of every live lane: precondition, sigma (the ring
        // GEMMs of all lanes in grouped launches), CGS2, Givens.  With use_graph
        // (and a plain preconditioner) it is captured once per window shape --
        // when that shape repeats, so every buffer is already sized and the
        // capture holds kernels only -- and replayed afterwards.
        if (graphable && graph_gen != alloc_generation()) {  // a buffer moved: drop stale graphs
          for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
          graphs.clear();
          seen.clear();
          graph_gen = alloc_generation();
        }
        for (int b = 0; b < nb; ++b) {
        ++n_iter;
        for (Lane* L : live) n_plane_iter += int64_t(L->active.size());
        if (!graphable) {
          iteration(live, s);
        } else {
          auto it = graphs.find(key);
          if (it != graphs.end()) {
            GFCC_HIP(hipGraphLaunch(it->second, s));
            lanes[0].c->prof["graph_replay"].count += 1;
          } else if (seen.count(key)) {
            // Record on a library stream: the caller's stream may be the legacy
            // default stream, which cannot be captured.  Recording executes
            // nothing; the graph is launched on the caller's stream.
            if (!cap.s) GFCC_HIP(hipStreamCreateWithFlags(&cap.s, hipStreamNonBlocking));
            hipGraph_t gr = nullptr;
            const uint64_t gen0 = alloc_generation();
            GFCC_HIP(hipStreamBeginCapture(cap.s, hipStreamCaptureModeThreadLocal));
            try {
              iteration(live, cap.s);
            } catch (...) {
              if (hipStreamEndCapture(cap.s, &gr) == hipSuccess && gr) (void)hipGraphDestroy(gr);
              (void)hipGetLastError();
              throw;
            }
            GFCC_HIP(hipStreamEndCapture(cap.s, &gr));
            if (alloc_generation() != gen0) {
              (void)hipGraphDestroy(gr);
              throw Error{GFCC_E_STATE, "allocation during graph capture"};
            }
            hipGraphExec_t ex;
            const hipError_t ie = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
            (void)hipGraphDestroy(gr);
            GFCC_HIP(ie);
            graphs[key] = ex;
            lanes[0].c->prof["graph_capture"].count += 1;
            GFCC_HIP(hipGraphLaunch(ex, s));
          } else {
            seen.insert(key);
            iteration(live, s);
          }
        }
        }
        // one copy of every lane's flags, Krylov steps and residual estimates, one synchronisation
        for (Lane* L : live)
          GFCC_HIP(hipMemcpyAsync(L->hstat.p, L->d_stat.p, size_t(L->B) * 16, hipMemcpyDeviceToHost, s));
        sync(s);
        ++n_loop_sync;
        for (Lane* L : live) {
          const int* hf = L->hstat.as<int>();
          const int* hk = hf + L->B;
          const double* hr = reinterpret_cast<const double*>(hf + 2 * L->B);
          std::vector<int> still;
          for (size_t i = 0; i < L->active.size(); ++i) {
            const int sl = L->active[i];
            HostSlot& h = L->hs[size_t(sl)];
            const int dk = hk[i] - h.k;  // iterations the slot ran in this burst
            if (dk > 0 && hr[i] > 0.0 && hr[i] < h.res && h.res > 0.0)
              h.lrate = std::log(hr[i] / h.res) / double(dk);
            h.res = hr[i];
            h.iters += dk;
            h.k = hk[i];
            if (hf[i] == 3) h.nonfinite = true;
            if (hf[i] != 0 || h.iters >= opts->max_iter)
              L->pending.push_back(sl);
            else
              still.push_back(sl);
          }
          L->active.swap(still);
        }
      }
      // finish cycles in groups: wait until half of a lane's live slots are
      // pending (slots advance in near lock-step, so this costs little
      // latency) so the FP64 true-residual sigma runs on a wide batch; when
      // every still active slot is predicted to stop within two iterations,
      // wait for them too (at most two iterations), so that they do not need
      // a true-residual sigma of their own on a few planes
      for (auto& L : lanes) {
        if (L.pending.empty()) continue;
        if (!L.active.empty() && L.pending.size() * 2 < L.active.size() + L.pending.size()) continue;
        if (!L.active.empty() && L.defer < 2 && all_stop_soon(L, 2)) {
          ++L.defer;
          continue;
        }
        L.defer = 0;
        finish(L);
      }
    }
    sync(s);
    gfcc_ctx* c0 = lanes[0].c;
    c0->prof["host_sync"].count += n_sync;
    c0->prof["loop_sync"].count += n_loop_sync;
    c0->prof["inner_iter"].count += n_iter;
    c0->prof["slot_iter"].count += n_plane_iter;
  }

  // every active slot of the lane stops its cycle within n more iterations (by its predicted
  // convergence, its restart length or its iteration budget)
  bool all_stop_soon(const Lane& L, int n) const {
    for (int sl : L.active) {
      const HostSlot& h = L.hs[size_t(sl)];
      if (m - h.k <= n || opts->max_iter - h.iters <= n) continue;
      if (!(h.lrate < 0.0)) return false;
      if (h.res > h.ctol && std::log(h.ctol / h.res) / h.lrate > double(n)) return false;
    }
    return true;
  }

  // Inner iterations to run before the next host synchronisation.  A slot whose
  // cycle stops inside the run is frozen on the device (its kernels return at
  // once; its planes of the batched sigma are computed and ignored), so the
  // length trades idle sigma work against synchronisations; it never passes a
  // slot's iteration budget.  Automatic lengths use each slot's predicted
  // iterations to its cycle target (from the observed decrease of its residual
  // estimate, capped by the restart length).  Where an iteration is short (the
  // estimated sigma time of the window under 2 ms, so that a synchronisation
  // is a visible share of it) the run goes on until half of a lane's slots are
  // predicted to stop -- the point where cycle finishing starts anyway; where
  // it is long, it ends at 85% of the first slot's prediction.
  int burst(const std::vector<Lane*>& live) const {
    const int se = opts->sync_every;
    if (se == 1 || use_mlp) return 1;
    for (Lane* L : live)
      if (L->c->prof_on) return 1;  // per-iteration traffic accounting needs every step's k
    int hard = 1 << 20;  // iteration budgets
    for (Lane* L : live)
      for (int sl : L->active) hard = std::min(hard, opts->max_iter - L->hs[size_t(sl)].iters);
    if (se > 1) return std::max(1, std::min(se, hard));
    const double rate = prec == GFCC_FP64 ? 50e12 : (prec == GFCC_FP32_IR ? 100e12 : 400e12);
    double t_est = 0.0;
    for (Lane* L : live) {
      const gfcc_ctx* c = L->c;
      const double per_plane = double(c->Dp) * (6.0 * double(c->ov) + (c->sector == 1 ? 2.0 * c->v * c->v : 0.0));
      t_est += 2.0 * double(L->active.size()) * per_plane / rate;
    }
    const bool short_iter = t_est < 2e-3;
    int S = 16;
    for (Lane* L : live) {
      std::vector<int> n;
      for (int sl : L->active) {
        const HostSlot& h = L->hs[size_t(sl)];
        int pred = short_iter ? 6 : 2;  // no rate observed yet
        if (h.lrate < 0.0)
          pred = h.res > h.ctol ? int(std::ceil(std::log(h.ctol / h.res) / h.lrate)) : 1;
        n.push_back(std::max(1, std::min(pred, m - h.k)));
      }
      std::sort(n.begin(), n.end());
      if (short_iter) {
        // slots still to stop before half of the lane's live slots are pending
        const size_t tot = L->active.size() + L->pending.size();
        const size_t need = (tot + 1) / 2 > L->pending.size() ? (tot + 1) / 2 - L->pending.size() : 1;
        S = std::min(S, n[std::min(need, n.size()) - 1]);
      } else {
        S = std::min(S, std::max(1, int(0.85 * n[0])));
      }
    }
    return std::max(1, std::min(S, hard));
  }
};

BatchRun make_run(const int64_t* p, const double* omega, double eta, int64_t nq, const int64_t* q,
                  const gfcc_solve_opts* opts, double* G, double* Xout, gfcc_rhs_info* info, hipStream_t s,
                  PairRec* rec) {
  BatchRun R{p, omega, eta, nq, q, opts, G, Xout, info, rec, s};
  R.m = std::min<int>(opts->restart, MAXM);
  R.prec = opts->precision;
  R.use_mlp = opts->precond == GFCC_PC_MLP;
  R.mode = R.use_mlp ? GFCC_PC_JACOBI : opts->precond;  // Jacobi is also the MLP fallback
  R.flex = R.use_mlp ? 1 : 0;
  R.tol = opts->tol;
  R.rtol_lp = (R.prec == GFCC_FP64) ? 0.0
              : (opts->ir_inner_rtol > 0.0 ? opts->ir_inner_rtol : lp_cycle_rtol(R.prec));
  return R;
}

double slot_bytes(const gfcc_ctx* c, int m, int flex) {
  return double(m + 2 + (flex ? m : 0)) * 2.0 * double(c->Dp) * 8.0 + 6.0 * 2.0 * double(c->Dp) * 8.0;
}

}  // namespace

void solve_batch(gfcc_ctx* c, int64_t nrhs, const int64_t* p, const double* omega, double eta, int64_t nq,
                 const int64_t* q, const gfcc_solve_opts* opts, double* G, double* Xout, gfcc_rhs_info* info,
                 hipStream_t s, bool* all_converged, PairRec* rec) {
  const bool use_mlp = opts->precond == GFCC_PC_MLP;
  GFCC_CHECK(!use_mlp || (c->mlp && c->mlp->trained), GFCC_E_STATE,
             "GFCC_PC_MLP needs trained or loaded network weights");
  for (int64_t r = 0; r < nrhs; ++r) info[r] = gfcc_rhs_info{1, 0, 0, 0, 0.0};
  BatchRun R = make_run(p, omega, eta, nq, q, opts, G, Xout, info, s, rec);
  int B = opts->batch > 0 ? opts->batch : 0;
  // reduced-precision operands first, so that the window is sized against what is left
  if (R.prec != GFCC_FP64) build_lowprec(c, lowp_index(R.prec), s);
  if (B == 0) {
    size_t freeb = 0, totalb = 0;
    GFCC_HIP(hipMemGetInfo(&freeb, &totalb));
    const int64_t fit = int64_t(0.8 * double(freeb) / slot_bytes(c, R.m, R.flex));
    B = int(std::max<int64_t>(1, std::min<int64_t>({fit, 512, nrhs})));
  }
  std::vector<Lane> lanes(1);
  lanes[0].c = c;
  lanes[0].B = int(std::min<int64_t>(B, nrhs));
  lanes[0].rows.resize(static_cast<size_t>(nrhs));
  for (int64_t r = 0; r < nrhs; ++r) lanes[0].rows[size_t(r)] = r;
  R.run(lanes, nrhs);
  *all_converged = R.ok_all;
}

// Right-hand sides of several systems in one persistent loop: one lane per
// system, the window split in proportion to each system's right-hand sides.
void solve_multi(int nsys, gfcc_ctx* const* ctxs, int64_t nrhs, const int32_t* sys, const int64_t* p,
                 const double* omega, double eta, int64_t nq, const int64_t* q, const gfcc_solve_opts* opts,
                 double* G, gfcc_rhs_info* info, hipStream_t s, bool* all_converged) {
  for (int64_t r = 0; r < nrhs; ++r) info[r] = gfcc_rhs_info{1, 0, 0, 0, 0.0};
  BatchRun R = make_run(p, omega, eta, nq, q, opts, G, nullptr, info, s, nullptr);
  R.sysv = sys;
  std::vector<Lane> lanes(static_cast<size_t>(nsys));
  for (int k = 0; k < nsys; ++k) lanes[size_t(k)].c = ctxs[k];
  for (int64_t r = 0; r < nrhs; ++r) lanes[size_t(sys[r])].rows.push_back(r);
  std::vector<Lane> used;
  for (auto& L : lanes)
    if (!L.rows.empty()) used.push_back(std::move(L));
  if (used.empty()) {
    *all_converged = true;
    return;
  }
  int64_t Btot = opts->batch > 0 ? opts->batch : std::min<int64_t>(nrhs, 128 * int64_t(used.size()));
  if (R.prec != GFCC_FP64)
    for (auto& L : used) build_lowprec(L.c, lowp_index(R.prec), s);
  size_t freeb = 0, totalb = 0;
  GFCC_HIP(hipMemGetInfo(&freeb, &totalb));
  for (;;) {  // window share of each system ~ its right-hand sides, within half of free memory
    double bytes = 0.0;
    for (auto& L : used) {
      L.B = int(std::max<int64_t>(1, std::min<int64_t>(int64_t(L.rows.size()),
                                                        int64_t(double(Btot) * double(L.rows.size()) / double(nrhs)))));
      bytes += double(L.B) * slot_bytes(L.c, R.m, R.flex);
    }
    if (bytes <= 0.5 * double(freeb) || Btot <= int64_t(used.size())) break;
    Btot = std::max<int64_t>(int64_t(used.size()), Btot * 3 / 4);
  }
  R.run(used, nrhs);
  *all_converged = R.ok_all;
}

}  // namespace gfcc

// sigma = Hbar_N x for a batch of vectors (the per-iteration O(o^3 v^2) work
// of the GFCCSD linear solver, paper: GFCC Workflow and Bottlenecks, Algorithm 1 singles and doubles).
//
// Closed-shell spin-adapted IP-EOM form, r1[i], r2[i,j,a]:
//   s1[i]     = -sum_m Foo[m,i] r1[m] + sum_me Fov[m,e](2 r2[i,m,e] - r2[m,i,e])
//               - sum_mne (2 Wooov[m,n,i,e] - Wooov[n,m,i,e]) r2[m,n,e]
//   s2[i,j,a] = -sum_m Wovoo[m,a,i,j] r1[m] + sum_e Fvv[a,e] r2[i,j,e]
//               - sum_m (Foo[m,i] r2[m,j,a] + Foo[m,j] r2[i,m,a]) + sum_mn Woooo[m,n,i,j] r2[m,n,a]
//               + sum_me (2 Wovvo[m,a,e,j] - Wovov[m,a,j,e]) r2[i,m,e]
//               - sum_me Wovvo[m,a,e,j] r2[m,i,e] - sum_me Wovov[m,a,i,e] r2[m,j,e]
//               - sum_e z_e t2[i,j,e,a],   z_e = sum_mnf (2(me|nf) - (mf|ne)) r2[m,n,f]
// Hbar_N is real; a complex vector is two real planes, so every term is a
// real GEMM whose N dimension runs over (vector, re/im, index).
//
// The three ring terms are the hot spot (12 o^3 v^2 flops per complex vector):
//   P1a: s2[(p,i)][(j,a)]  = R [(p,i)][(m,e)] . X1 [(j,a)][(m,e)]^T   (R = r2 rows)
//   P1b: s2[(p,i)][(j,a)] -= RT[(p,i)][(m,e)] . Wvo[(j,a)][(m,e)]^T   (RT[i][m][e] = r2[m][i][e])
//   P2 : s2[(p,j)][(i,a)] -= RT[(p,j)][(m,e)] . Wov[(i,a)][(m,e)]^T   (scattered store)
// In FP32/BF16 mode these three and the hole-hole ladder and z contraction
// read reduced-precision copies; the one-body terms stay FP64.
#include <algorithm>
#include <cstring>
#include <string>

#include "ctx.h"

namespace gfcc {

template <typename T> __device__ __forceinline__ T cvt(double x);
template <> __device__ __forceinline__ double cvt<double>(double x) { return x; }
template <> __device__ __forceinline__ float cvt<float>(double x) { return float(x); }
template <> __device__ __forceinline__ __bf16 cvt<__bf16>(double x) { return __bf16(float(x)); }

// RT[p][i*ov + m*v + e] = x[p*Dp + o_pad + m*ov + i*v + e]   (and R when R != nullptr)
// and the FP64 diagonal one-body part  y2[p][t] = d1b[t] x2[p][t]  (initialises y2)
template <typename T>
__global__ void make_rt_kernel(const double* __restrict__ x, T* __restrict__ RT, T* __restrict__ R,
                               double* __restrict__ y, const double* __restrict__ d1b, int64_t o, int64_t v,
                               int64_t Dp, int64_t o_pad, int64_t ps) {
  const int64_t oov = o * o * v, ov = o * v;
  const int64_t p = blockIdx.y;
  const double* xp = x + p * Dp + o_pad;
  double* yp = y + p * Dp + o_pad;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < oov; t += int64_t(gridDim.x) * blockDim.x) {
    const int64_t e = t % v, m = (t / v) % o, i = t / ov;  // output order [i][m][e]
    RT[p * ps + t] = cvt<T>(xp[m * ov + i * v + e]);
    const double xt = xp[t];
    if (R) R[p * ps + t] = cvt<T>(xt);
    yp[t] = d1b[t] * xt;
  }
}

// Ra[p][a][(m,n)] = x[p*Dp + o_pad + (m,n)*v + a]  (row stride op2), LDS-tiled transpose
template <typename T>
__global__ void make_ra_kernel(const double* __restrict__ x, T* __restrict__ Ra, int64_t oo, int64_t v,
                               int64_t Dp, int64_t o_pad, int64_t op2) {
  __shared__ double tile[32][33];
  const int64_t p = blockIdx.z;
  const int64_t r0 = int64_t(blockIdx.x) * 32, c0 = int64_t(blockIdx.y) * 32;  // rows (m,n), cols a
  const double* xp = x + p * Dp + o_pad;
  for (int k = threadIdx.y; k < 32; k += 8) {
    const int64_t r = r0 + k, cc = c0 + threadIdx.x;
    tile[k][threadIdx.x] = (r < oo && cc < v) ? xp[r * v + cc] : 0.0;
  }
  __syncthreads();
  for (int k = threadIdx.y; k < 32; k += 8) {
    const int64_t a = c0 + k, r = r0 + threadIdx.x;
    if (a < v && r < oo) Ra[(p * v + a) * op2 + r] = cvt<T>(tile[threadIdx.x][k]);
  }
}

static unsigned blocks_for(int64_t n) {
  return unsigned(std::min<int64_t>(std::max<int64_t>((n + 255) / 256, 1), 4096));
}

// A[p][k] of the fused three-body + 2h1p<-1h GEMM: [z_p (v) | 0 | r1_p (o) | 0], row stride ktw
template <typename T>
__global__ void make_zr_kernel(const double* __restrict__ z, const double* __restrict__ x, T* __restrict__ A,
                               int64_t v, int64_t vp, int64_t o, int64_t ktw, int64_t Dp) {
  const int64_t p = blockIdx.x;
  for (int64_t k = threadIdx.x; k < ktw; k += blockDim.x) {
    double val = 0.0;
    if (k < v)
      val = z[p * vp + k];
    else if (k >= vp && k < vp + o)
      val = x[p * Dp + (k - vp)];
    A[p * ktw + k] = cvt<T>(val);
  }
}

template <typename T>
static void make_operands(gfcc_ctx* c, int64_t P, const double* x, T* RT, T* R, T* Ra, int64_t ps, double* y,
                          hipStream_t s) {
  const int64_t oov = c->oov;
  hipLaunchKernelGGL((make_rt_kernel<T>), dim3(std::min<int64_t>((oov + 255) / 256, 1024), unsigned(P)),
                     dim3(256), 0, s, x, RT, R, y, c->d1b.as<double>(), c->o, c->v, c->Dp, c->o_pad, ps);
  GFCC_HIP(hipGetLastError());
  dim3 g(unsigned((c->oo + 31) / 32), unsigned((c->v + 31) / 32), unsigned(P));
  hipLaunchKernelGGL((make_ra_kernel<T>), g, dim3(32, 8), 0, s, x, Ra, c->oo, c->v, c->Dp, c->o_pad, c->op2);
  GFCC_HIP(hipGetLastError());
}

// phases of one sigma: operand copies, the three ring GEMMs, everything else
enum : int { PH_OPS = 1, PH_RING = 2, PH_REST = 4, PH_ALL = 7 };

// With ring_out != nullptr the ring phase returns its three GEMMs (and tile)
// instead of launching them, for a grouped launch over several systems.
static void sigma_impl(gfcc_ctx* c, int64_t P, const double* x, double* y, gfcc_precision prec, hipStream_t s,
                       int phases, GemmArgs* ring_out, int* ring_cfg) {
  if (P <= 0) return;
  const int64_t o = c->o, v = c->v, ov = c->ov, oo = c->oo, oov = c->oov;
  const int64_t Dp = c->Dp, op = c->o_pad, kp = c->kp;
  const bool lowp = prec != GFCC_FP64;
  const int li = (prec == GFCC_BF16_IR) ? 1 : 0;
  const Prec rp = !lowp ? Prec::F64 : (li ? Prec::BF16 : Prec::F32);
  const int64_t esz = !lowp ? 8 : (li ? 2 : 4);
  if (lowp) build_lowprec(c, li, s);
  const int64_t ps = round_up(oov, 8);  // plane stride of operand copies
  c->ws_RT.ensure(size_t(P * ps * esz), s);
  c->ws_Ra.ensure(size_t(P * v * c->op2 * esz), s);
  if (lowp) c->ws_R.ensure(size_t(P * ps * esz), s);
  c->ws_z.ensure(size_t(P * c->vp * 8), s);

  const bool whole = phases == PH_ALL;
  if (whole) prof_begin(c, "sigma", s);
  if (phases & PH_OPS) {
    switch (rp) {
      case Prec::F64:
        make_operands<double>(c, P, x, c->ws_RT.as<double>(), nullptr, c->ws_Ra.as<double>(), ps, y, s);
        break;
      case Prec::F32:
        make_operands<float>(c, P, x, c->ws_RT.as<float>(), c->ws_R.as<float>(), c->ws_Ra.as<float>(), ps, y, s);
        break;
      case Prec::BF16:
        make_operands<__bf16>(c, P, x, c->ws_RT.as<__bf16>(), c->ws_R.as<__bf16>(), c->ws_Ra.as<__bf16>(), ps, y,
                               s);
        break;
    }
  }
  const auto& L = c->lp[li];
  const void* X1 = lowp ? L.X1.p : c->X1.p;
  const void* Wvo = lowp ? L.Wvo.p : c->Wvo.p;
  const void* Wov = lowp ? L.Wov.p : c->Wov.p;
  const void* W4T = lowp ? L.W4T.p : c->W4T.p;
  const void* Zm = lowp ? L.Zm.p : c->Zm.p;
  const double sX1 = lowp ? 1.0 / L.sX1 : 1.0, sWvo = lowp ? 1.0 / L.sWvo : 1.0;
  const double sWov = lowp ? 1.0 / L.sWov : 1.0, sW4T = lowp ? 1.0 / L.sW4T : 1.0;
  const double sZm = lowp ? 1.0 / L.sZm : 1.0;

  const double ring_flops = 2.0 * double(P) * double(o) * double(ov) * double(ov);
  const char* ring_name = !lowp ? "ring_gemm_fp64" : (li ? "ring_gemm_bf16" : "ring_gemm_fp32");
  const double ring_bytes = double(ov) * double(kp) * esz + 2.0 * double(P) * double(o) * double(ov) * (esz + 8.0);

  // ---- ring terms
  if (phases & PH_RING) {
    GemmArgs g;
    g.M = P * o;
    g.N = ov;
    g.K = ov;
    g.C = y + op;
    g.cm = two(o, Dp, ov);
    g.cn = lin(1);
    const int cfg = tuned_cfg(c, rp, g.M, g.N, g.K);
    // P1a
    if (lowp) {
      g.A = c->ws_R.p;
      g.am = two(o, ps, ov);
    } else {
      g.A = x + op;
      g.am = two(o, Dp, ov);
    }
    g.B = X1;
    g.bm = lin(kp);
    g.alpha = sX1;
    g.beta = 1.0;  // y2 holds the diagonal one-body part
    auto run = [&](int k) {
      if (ring_out) {
        ring_out[k] = g;
        *ring_cfg = cfg;
        return;
      }
      prof_begin(c, ring_name, s);
      gemm(rp, g, cfg, s);
      prof_end(c, ring_name, s, ring_flops, ring_bytes);
    };
    run(0);
    // P1b
    g.A = c->ws_RT.p;
    g.am = two(o, ps, ov);
    g.B = Wvo;
    g.alpha = -sWvo;
    g.beta = 1.0;
    run(1);
    // P2: rows (p, j), cols (i, a) -> s2[p][i][j][a]
    g.B = Wov;
    g.alpha = -sWov;
    g.cm = two(o, Dp, v);
    g.cn = two(v, ov, 1);
    run(2);
  }
  if (!(phases & PH_REST)) return;
  // ---- hole-hole ladder: s2[p][(i,j)][a] += sum_(mn) W4T[(i,j)][(m,n)] Ra[(p,a)][(m,n)]
  {
    GemmArgs g;
    g.A = W4T;
    g.am = lin(c->op2);
    g.B = c->ws_Ra.p;
    g.bm = lin(c->op2);
    g.M = oo;
    g.N = P * v;
    g.K = oo;
    g.C = y + op;
    g.cm = lin(v);
    g.cn = two(v, Dp, 1);
    g.alpha = sW4T;
    g.beta = 1.0;
    gemm(rp, g, tuned_cfg(c, rp, g.M, g.N, g.K), s);
  }
  // ---- three-body: z[p][e] = sum_(mnf) Zm[e][(m,n,f)] r2[p][(m,n,f)];  s2 -= z . t2
  {
    GemmArgs g;
    if (lowp) {
      g.A = c->ws_R.p;
      g.am = lin(ps);
    } else {
      g.A = x + op;
      g.am = lin(Dp);
    }
    g.B = Zm;
    g.bm = lin(c->ldz);
    g.M = P;
    g.N = v;
    g.K = oov;
    g.C = c->ws_z.as<double>();
    g.cm = lin(c->vp);
    g.cn = lin(1);
    g.alpha = sZm;
    g.beta = 0.0;
    gemm_auto(rp, g, c->scr, 0, s);
  }
  // ---- three-body second half and 2h1p <- 1h in one GEMM:
  //      s2[p][(i,j,a)] -= sum_e z[p][e] t2[i,j,e,a] + sum_m r1[p][m] Wovoo[m,a,i,j]
  {
    const int64_t ktw = c->ktw;
    c->ws_zr.ensure(size_t(P * ktw * esz), s);
    switch (rp) {
      case Prec::F64:
        hipLaunchKernelGGL((make_zr_kernel<double>), dim3(unsigned(P)), dim3(256), 0, s, c->ws_z.as<double>(), x,
                           c->ws_zr.as<double>(), v, c->vp, o, ktw, Dp);
        break;
      case Prec::F32:
        hipLaunchKernelGGL((make_zr_kernel<float>), dim3(unsigned(P)), dim3(256), 0, s, c->ws_z.as<double>(), x,
                           c->ws_zr.as<float>(), v, c->vp, o, ktw, Dp);
        break;
      case Prec::BF16:
        hipLaunchKernelGGL((make_zr_kernel<__bf16>), dim3(unsigned(P)), dim3(256), 0, s, c->ws_z.as<double>(), x,
                           c->ws_zr.as<__bf16>(), v, c->vp, o, ktw, Dp);
        break;
    }
    GFCC_HIP(hipGetLastError());
    GemmArgs h;
    h.A = c->ws_zr.p;
    h.am = lin(ktw);
    h.B = lowp ? L.TW.p : c->TW.p;
    h.bm = lin(ktw);
    h.M = P;
    h.N = oov;
    h.K = ktw;
    h.C = y + op;
    h.cm = lin(Dp);
    h.cn = lin(1);
    h.alpha = lowp ? -1.0 / L.sTW : -1.0;
    h.beta = 1.0;
    gemm(rp, h, tuned_cfg(c, rp, h.M, h.N, h.K), s);
  }
  // ---- 1h rows: s1[p][i] = sum_k x[p][k] Uop[i][k]   (FP64)
  {
    GemmArgs g;
    g.A = x;
    g.am = lin(Dp);
    g.B = c->Uop.p;
    g.bm = lin(Dp);
    g.M = P;
    g.N = o;
    g.K = Dp;
    g.C = y;
    g.cm = lin(Dp);
    g.cn = lin(1);
    g.alpha = 1.0;
    g.beta = 0.0;
    gemm_auto(Prec::F64, g, c->scr, 0, s);
  }
  const double total_flops = 3.0 * ring_flops + 2.0 * double(P) * (double(oo) * oo * v + 2.0 * oov * v +
                                                                    double(oov) * v + double(oov) * o +
                                                                    2.0 * double(oov) * o + double(Dp) * o);
  if (whole) prof_end(c, "sigma", s, total_flops, 0.0);
}

void sigma_planes(gfcc_ctx* c, int64_t P, const double* x, double* y, gfcc_precision prec, hipStream_t s) {
  sigma_impl(c, P, x, y, prec, s, PH_ALL, nullptr, nullptr);
}

// Several systems: operand copies per system, each ring term of all systems in
// one grouped launch (tile of the largest system), the remaining terms per system.
void sigma_group(const SigmaJob* jobs, int nj, gfcc_precision prec, hipStream_t s) {
  int live = 0;
  for (int j = 0; j < nj; ++j) live += jobs[j].P > 0 ? 1 : 0;
  if (live <= 1 || nj > MAX_GEMM_GROUPS) {
    for (int j = 0; j < nj; ++j) sigma_planes(jobs[j].c, jobs[j].P, jobs[j].x, jobs[j].y, prec, s);
    return;
  }
  const Prec rp = prec == GFCC_FP64 ? Prec::F64 : (prec == GFCC_BF16_IR ? Prec::BF16 : Prec::F32);
  GemmArgs ring[3][MAX_GEMM_GROUPS];
  int ng = 0, cfg = 0;
  double best = -1.0;
  for (int j = 0; j < nj; ++j) {
    const SigmaJob& J = jobs[j];
    if (J.P <= 0) continue;
    sigma_impl(J.c, J.P, J.x, J.y, prec, s, PH_OPS, nullptr, nullptr);
    GemmArgs g3[3];
    int cj = 0;
    sigma_impl(J.c, J.P, J.x, J.y, prec, s, PH_RING, g3, &cj);
    for (int t = 0; t < 3; ++t) ring[t][ng] = g3[t];
    const double size = double(g3[0].M) * double(g3[0].N);
    if (size > best) {
      best = size;
      cfg = cj;
    }
    ++ng;
  }
  for (int t = 0; t < 3; ++t) gemm_grouped(rp, ring[t], ng, cfg, s);
  for (int j = 0; j < nj; ++j)
    if (jobs[j].P > 0) sigma_impl(jobs[j].c, jobs[j].P, jobs[j].x, jobs[j].y, prec, s, PH_REST, nullptr, nullptr);
}

// ------------------------------------------------------------------ layout conversions

__global__ void to_planes_kernel(const double* __restrict__ xi, double* __restrict__ pl, int64_t nb, int64_t D,
                                 int64_t Dp, int64_t o, int64_t o_pad) {
  const int64_t b = blockIdx.y;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < D; t += int64_t(gridDim.x) * blockDim.x) {
    const int64_t dst = (t < o) ? t : (t - o + o_pad);
    pl[(2 * b) * Dp + dst] = xi[(b * D + t) * 2];
    pl[(2 * b + 1) * Dp + dst] = xi[(b * D + t) * 2 + 1];
  }
}

__global__ void from_planes_kernel(const double* __restrict__ pl, double* __restrict__ xi, int64_t nb, int64_t D,
                                   int64_t Dp, int64_t o, int64_t o_pad) {
  const int64_t b = blockIdx.y;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < D; t += int64_t(gridDim.x) * blockDim.x) {
    const int64_t src = (t < o) ? t : (t - o + o_pad);
    xi[(b * D + t) * 2] = pl[(2 * b) * Dp + src];
    xi[(b * D + t) * 2 + 1] = pl[(2 * b + 1) * Dp + src];
  }
}

void to_planes(gfcc_ctx* c, int64_t nb, const double* xi, double* planes, hipStream_t s) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(to_planes_kernel, dim3(blocks_for(c->D), unsigned(nb)), dim3(256), 0, s, xi, planes, nb,
                     c->D, c->Dp, c->o, c->o_pad);
  GFCC_HIP(hipGetLastError());
}

void from_planes(gfcc_ctx* c, int64_t nb, const double* planes, double* xi, hipStream_t s) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(from_planes_kernel, dim3(blocks_for(c->D), unsigned(nb)), dim3(256), 0, s, planes, xi, nb,
                     c->D, c->Dp, c->o, c->o_pad);
  GFCC_HIP(hipGetLastError());
}

// Right-hand sides b_p = abar_p|Phi> on the 1h + 2h1p space as real planes
// (Theory section, the linear system for X_p): occupied p gives the unit vector
// e_p; virtual p (a = p - o) gives [a_p, T]|Phi>: b(1h)_i = t_i^a and, in the
// doublet basis, b(2h1p)_ijb = t_ij^ab.
__global__ void rhs_rows_kernel(const int64_t* __restrict__ orb, const double* __restrict__ t1,
                                const double* __restrict__ TW, int64_t ktw, double* __restrict__ out, int64_t o,
                                int64_t v, int64_t o_pad, int64_t Dp) {
  const int64_t r = blockIdx.y;
  const int64_t p = orb[r];
  const int64_t oov = o * o * v;
  double* row = out + r * Dp;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < Dp; t += int64_t(gridDim.x) * blockDim.x) {
    double val = 0.0;
    if (p < o) {
      val = (t == p) ? 1.0 : 0.0;
    } else {
      const int64_t a = p - o;
      if (t < o)
        val = t1[t * v + a];
      else if (t >= o_pad && t - o_pad < oov)
        val = TW[(t - o_pad) * ktw + a];  // t2[i, j, a, b] at row (i, j, b)
    }
    row[t] = val;
  }
}

// Left vectors c_q = <Phi|(1 + Lambda) abar_q^+ as real planes: occupied q from the
// rows built with the intermediates; virtual q (a = q - o): abar_q^+ = a_q^+ and
// c(1h)_i = l_i^a, c(2h1p)_klc = 2 l_kl^ac - l_kl^ca.
__global__ void left_rows_kernel(const int64_t* __restrict__ orb, const double* __restrict__ left_occ,
                                 const double* __restrict__ l1, const double* __restrict__ l2,
                                 const double* __restrict__ TW, int64_t ktw, double* __restrict__ out, int64_t o,
                                 int64_t v, int64_t o_pad, int64_t Dp) {
  const int64_t r = blockIdx.y;
  const int64_t q = orb[r];
  const int64_t oov = o * o * v;
  double* row = out + r * Dp;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < Dp; t += int64_t(gridDim.x) * blockDim.x) {
    double val = 0.0;
    if (q < o) {
      val = left_occ[q * Dp + t];
    } else {
      const int64_t a = q - o;
      if (t < o) {
        val = l1[t * v + a];
      } else if (t >= o_pad && t - o_pad < oov) {
        const int64_t idx = t - o_pad, kl = idx / v, cc = idx % v;  // (k, l, c)
        if (l2)
          val = 2.0 * l2[(kl * v + a) * v + cc] - l2[(kl * v + cc) * v + a];
        else  // l2 = t2: l2[k, l, a, c] at TW row (k, l, c), column a
          val = 2.0 * TW[idx * ktw + a] - TW[(kl * v + a) * ktw + cc];
      }
    }
    row[t] = val;
  }
}

void make_rhs_rows(gfcc_ctx* c, int64_t n, const int64_t* orb_dev, double* out, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(rhs_rows_kernel, dim3(blocks_for(c->Dp), unsigned(n)), dim3(256), 0, s, orb_dev,
                     c->t1c.as<double>(), c->TW.as<double>(), c->ktw, out, c->o, c->v, c->o_pad, c->Dp);
  GFCC_HIP(hipGetLastError());
}

void make_left_rows(gfcc_ctx* c, int64_t n, const int64_t* orb_dev, double* out, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(left_rows_kernel, dim3(blocks_for(c->Dp), unsigned(n)), dim3(256), 0, s, orb_dev,
                     c->left.as<double>(), c->l1c.as<double>(), c->l2c.p ? c->l2c.as<double>() : nullptr,
                     c->TW.as<double>(), c->ktw, out, c->o, c->v, c->o_pad, c->Dp);
  GFCC_HIP(hipGetLastError());
}

// Split-K partials (doubles) of the G product for nb vectors and nq left rows; 0 when
// the tile grid fills the GPU without splitting K.
int64_t greens_part_doubles(gfcc_ctx* c, int64_t nb, int64_t nq) {
  const int sl = splitk_slices(2 * nb, nq, c->Dp);
  return sl > 1 ? int64_t(sl) * 2 * nb * nq : 0;
}

// G[r][k] = rows[k] . x_r with caller-provided left rows [nq][Dp] and split-K
// partials (greens_part_doubles of them; nullptr when that is 0)
void greens_rows(gfcc_ctx* c, int64_t nb, const double* planes, int64_t nq, const double* rows, double* G,
                 double* part, hipStream_t s) {
  if (nb <= 0 || nq <= 0) return;
  GemmArgs g;
  g.A = planes;
  g.am = lin(c->Dp);
  g.B = rows;
  g.bm = lin(c->Dp);
  g.M = 2 * nb;
  g.N = nq;
  g.K = c->Dp;
  g.C = G;
  g.cm = two(2, 2 * nq, 1);
  g.cn = lin(2);
  g.alpha = 1.0;
  g.beta = 0.0;
  const int sl = splitk_slices(g.M, g.N, g.K);
  if (sl <= 1)
    gemm(Prec::F64, g, gemm_default_cfg(g.M, g.N, g.K), s);
  else
    gemm_splitk(Prec::F64, g, sl, part, s);
}

// G[r][k] = c_{q_k} . x_r  (re from plane 2r, im from plane 2r+1)
void greens_planes(gfcc_ctx* c, int64_t nb, const double* planes, int64_t nq, const int64_t* q_dev, double* G,
                   hipStream_t s) {
  if (nb <= 0 || nq <= 0) return;
  double* rows = c->scr.get(3, nq * c->Dp, s);
  make_left_rows(c, nq, q_dev, rows, s);
  GemmArgs g;
  g.A = planes;
  g.am = lin(c->Dp);
  g.B = rows;
  g.bm = lin(c->Dp);
  g.M = 2 * nb;
  g.N = nq;
  g.K = c->Dp;
  g.C = G;
  g.cm = two(2, 2 * nq, 1);
  g.cn = lin(2);
  g.alpha = 1.0;
  g.beta = 0.0;
  gemm_auto(Prec::F64, g, c->scr, 0, s);
}

// Spectral function (Theory section, trace of the imaginary part of the
// retarded G): A[k] = sgn(eta) / pi * sum_p Im G[p][k].  With the operator
// (omega + Hbar_N - i eta) and eta > 0 the poles give Im G_pp > 0, so the sign
// keeps A >= 0 for either sign of eta (G(omega, -eta) = conj G(omega, eta)).
__global__ void spectral_kernel(const double* __restrict__ G, int64_t np, int64_t ld, double scale,
                                double* __restrict__ A) {
  const int64_t k = blockIdx.x;
  double acc = 0.0;
  for (int64_t p = threadIdx.x; p < np; p += blockDim.x) acc += G[(p * ld + k) * 2 + 1];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) A[k] = scale * (red[0] + red[1] + red[2] + red[3]);
}

void spectral(int64_t np, int64_t nw, const double* G, int64_t ld, double eta, double* A, hipStream_t s) {
  if (nw <= 0) return;
  const double scale = (eta < 0.0 ? -1.0 : 1.0) / M_PI;
  hipLaunchKernelGGL(spectral_kernel, dim3(unsigned(nw)), dim3(256), 0, s, G, np, ld, scale, A);
  GFCC_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ timing

void prof_begin(gfcc_ctx* c, const char* name, hipStream_t s) {
  if (!c->prof_on) return;
  hipEvent_t a, b;
  GFCC_HIP(hipEventCreate(&a));
  GFCC_HIP(hipEventCreate(&b));
  GFCC_HIP(hipEventRecord(a, s));
  c->prof_events[name].push_back({a, b});
}

void prof_end(gfcc_ctx* c, const char* name, hipStream_t s, double flops, double bytes) {
  if (!c->prof_on) return;
  auto& v = c->prof_events[name];
  GFCC_CHECK(!v.empty(), GFCC_E_STATE, "prof_end without prof_begin");
  GFCC_HIP(hipEventRecord(v.back().second, s));
  c->prof_meta[name].push_back({flops, bytes});
  if (v.size() >= 4096) prof_collect(c);
}

void prof_collect(gfcc_ctx* c) {
  for (auto& kv : c->prof_events) {
    auto& meta = c->prof_meta[kv.first];
    auto& e = c->prof[kv.first];
    for (size_t k = 0; k < kv.second.size(); ++k) {
      GFCC_HIP(hipEventSynchronize(kv.second[k].second));
      float ms = 0.f;
      GFCC_HIP(hipEventElapsedTime(&ms, kv.second[k].first, kv.second[k].second));
      e.count += 1;
      e.ms += ms;
      if (k < meta.size()) {
        e.flops += meta[k].flops;
        e.bytes += meta[k].bytes;
      }
      (void)hipEventDestroy(kv.second[k].first);
      (void)hipEventDestroy(kv.second[k].second);
    }
    kv.second.clear();
    meta.clear();
  }
}

}  // namespace gfcc

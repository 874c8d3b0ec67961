// The advanced (electron-attached) term of the GFCCSD Green's function.
//
// Paper, Theory section: the second term of the Green's function,
//   G^EA_pq(omega) = <Phi|(1 + Lambda) abar_p Y_q|Phi>,
//   (omega - Hbar_N + i eta) Y_q |Phi> = abar_q^+ |Phi>,
// with Y_q expanded in one-particle a_a^+ and two-particle-one-hole a_a^+ a_b^+ a_j operators.
// The library runs it through the IP solver as (-omega - i eta + Hbar_N) Y_q = -abar_q^+|Phi>:
// the entry points negate omega and the right-hand-side rows carry the minus sign.
//
// Closed-shell spin-adapted basis (doublet), dimension v + o v^2:
//   y[a]                       coefficient of a^+_{a alpha}
//   y[v + (j v + a) v + b]     coefficient of a^+_{a alpha} a^+_{b beta} a_{j beta}
// (the same-spin part is y_jab - y_jba).  Planes hold the 1p block at [0, v) and the 2p1h block
// at [p1, p1 + o v^2), p1 = round8(v).
//
// Sigma as GEMMs over P planes (FP64 on MFMA):
//   1p   <- plane         Uop [v][Dp]: Fvv on 1p; 2 Wvovv[a,l,c,d] - Wvovv[a,l,d,c] with the Fov terms on 2p1h
//   2p1h <- 1p            Wvvvo (K = v)
//   2p1h <- 2p1h ring     rows (x,a) x [y[l,a,d] | y[l,c,a]] against [2Wovvo - Wovov | -Wovvo] (K = 2 ov),
//                         rows (x,b) x y[l,c,b] against -Wovov (K = ov); the one-body Foo/Fvv terms folded in
//   2p1h <- 2p1h ladder   rows (x,j) x y[j,c,d] against Wvvvv[(a,b)][(c,d)] (K = v^2, the dominant product)
//   2p1h <- 2p1h 3-body   z[x,k] = y . (2(kc|ld) - (kd|lc)), then -z . t2
//
// Building the blocks: Wvvvv factorises through the T1-dressed Cholesky vectors
// M_Q[a,c] = L_Q[a,c] - sum_k t_ka L_Q[k,c]: the bare and T1 parts of the ladder are
// sum_Q M_Q[a,c] M_Q[b,d] (the T1 T1 part of tau cancels against them), the rest is
// sum_kl t_kl^ab (kc|ld).  Wvovv = sum_Q M_Q[a,c] L_Q[l,d].
#include <cmath>

#include "ctx.h"

namespace gfcc {
namespace {

unsigned nblk(int64_t n) { return unsigned(std::min<int64_t>((n + 255) / 256, 65535)); }

// ------------------------------------------------------------------ build kernels

__global__ void add_eps_kernel(double* __restrict__ F, const double* __restrict__ eps, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) F[i * n + i] += eps[i];
}

// tau[i,j,a,b] = t2[i,j,a,b] + t1[i,a] t1[j,b];  ut[i,j,a,b] = 2 x[i,j,a,b] - x[i,j,b,a]
__global__ void tau_kernel(const double* __restrict__ t2, const double* __restrict__ t1, double* __restrict__ tau,
                           int64_t o, int64_t v) {
  const int64_t n = o * o * v * v;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n; t += int64_t(gridDim.x) * blockDim.x) {
    const int64_t b = t % v, a = (t / v) % v, j = (t / (v * v)) % o, i = t / (o * v * v);
    tau[t] = t2[t] + t1[i * v + a] * t1[j * v + b];
  }
}
__global__ void unsym_kernel(const double* __restrict__ x, double* __restrict__ ut, int64_t o, int64_t v) {
  const int64_t n = o * o * v * v;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n; t += int64_t(gridDim.x) * blockDim.x) {
    const int64_t b = t % v, a = (t / v) % v, ij = t / (v * v);
    ut[t] = 2.0 * x[t] - x[(ij * v + b) * v + a];
  }
}

// Uop[a][c] = Fvv[a,c];  Uop[a][p1 + (l,c,d)] += 2 d_ac Fov[l,d] - d_ad Fov[l,c]
__global__ void uop_fold_kernel(double* __restrict__ U, const double* __restrict__ Fvv, const double* __restrict__ Fov,
                                int64_t o, int64_t v, int64_t p1, int64_t Dp) {
  const int64_t a = blockIdx.y;
  double* u = U + a * Dp;
  const int64_t n = o * v * v;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n; t += int64_t(gridDim.x) * blockDim.x) {
    if (t < v) u[t] = Fvv[a * v + t];
    const int64_t d = t % v, cc = (t / v) % v, l = t / (v * v);
    double add = 0.0;
    if (cc == a) add += 2.0 * Fov[l * v + d];
    if (d == a) add -= Fov[l * v + cc];
    if (add != 0.0) u[p1 + t] += add;
  }
}

// ring[(j,b)][(l,d)] += d_bd (-Foo[l,j]) + d_lj Fvv[b,d];  ring2[(j,a)][(l,c)] += d_lj Fvv[a,c]
__global__ void ring_fold_kernel(double* __restrict__ R, double* __restrict__ R2, const double* __restrict__ Foo,
                                 const double* __restrict__ Fvv, int64_t o, int64_t v, int64_t kp) {
  const int64_t ov = o * v, n = ov * ov;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n; t += int64_t(gridDim.x) * blockDim.x) {
    const int64_t row = t / ov, col = t % ov;
    const int64_t j = row / v, b = row % v, l = col / v, d = col % v;
    double add = 0.0;
    if (d == b) add -= Foo[l * o + j];
    if (l == j) add += Fvv[b * v + d];
    if (add != 0.0) R[row * 2 * kp + col] += add;
    if (l == j) R2[row * kp + col] += Fvv[b * v + d];
  }
}

// exact diagonal of Hbar_N on 1p + 2p1h (padding 1.0)
__global__ void ea_diag_kernel(double* __restrict__ dg, const double* __restrict__ Fvv,
                               const double* __restrict__ lad, const double* __restrict__ R,
                               const double* __restrict__ R2, const double* __restrict__ zop,
                               const double* __restrict__ t2, int64_t o, int64_t v, int64_t p1, int64_t Dp,
                               int64_t kp, int64_t lv, int64_t n2p) {
  const int64_t vv = v * v, n2 = o * vv;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < Dp; t += int64_t(gridDim.x) * blockDim.x) {
    double d = 1.0;
    if (t < v) {
      d = Fvv[t * v + t];
    } else if (t >= p1 && t - p1 < n2) {
      const int64_t idx = t - p1, j = idx / vv, ab = idx % vv, a = ab / v, b = ab % v;
      d = lad[ab * lv + ab] + R[(j * v + b) * 2 * kp + j * v + b] + R2[(j * v + a) * kp + j * v + a];
      if (a == b) d += R[(j * v + b) * 2 * kp + kp + j * v + a];
      double tb = 0.0;
      for (int64_t k = 0; k < o; ++k) tb += zop[k * n2p + idx] * t2[k * n2 + idx];
      d -= tb;
    }
    dg[t] = d;
  }
}

// ------------------------------------------------------------------ sigma kernels

// R[(x,a)][(l,d)] = y[x][p1 + (l,a,d)],  R[(x,a)][kp + (l,c)] = y[x][p1 + (l,c,a)]; padding zero.
// T = _Float16: values multiplied by the device scale sc[0] on conversion.
template <typename T>
__global__ void ea_ring_operand_kernel(const double* __restrict__ x, T* __restrict__ R, int64_t o, int64_t v,
                                       int64_t p1, int64_t Dp, int64_t kp, const double* __restrict__ sc) {
  const int64_t row = blockIdx.x;  // (plane, a)
  const int64_t pl = row / v, a = row % v;
  const double* y = x + pl * Dp + p1;
  T* r = R + row * 2 * kp;
  const int64_t ov = o * v;
  const double sv = sc ? sc[0] : 1.0;
  for (int64_t t = threadIdx.x; t < kp; t += blockDim.x) {
    double u = 0.0, w = 0.0;
    if (t < ov) {
      const int64_t l = t / v, e = t % v;
      u = y[(l * v + a) * v + e];
      w = y[(l * v + e) * v + a];
    }
    r[t] = T(sv * u);
    r[kp + t] = T(sv * w);
  }
}

__global__ void fill_zero_kernel(double* __restrict__ p, int64_t n) {
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n; t += int64_t(gridDim.x) * blockDim.x)
    p[t] = 0.0;
}

// dst = f16(sc * src) over n elements (sc a device scalar)
__global__ void to_f16_scaled_kernel(const double* __restrict__ src, _Float16* __restrict__ dst, int64_t n,
                                     const double* __restrict__ sc) {
  const double sv = *sc;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n; t += int64_t(gridDim.x) * blockDim.x)
    dst[t] = _Float16(float(sv * src[t]));
}

// padding of output planes: [n1, p1) and [p1 + n2, Dp)
__global__ void zero_pads_kernel(double* __restrict__ y, int64_t n1, int64_t p1, int64_t n2, int64_t Dp) {
  double* yp = y + int64_t(blockIdx.y) * Dp;
  const int64_t w1 = p1 - n1, w2 = Dp - p1 - n2;
  for (int64_t t = threadIdx.x; t < w1 + w2; t += blockDim.x) yp[t < w1 ? n1 + t : p1 + n2 + (t - w1)] = 0.0;
}

// rows of the solved system: -abar_q^+|Phi>.  Occupied q = i: +t_i^c on 1p, +t_ij^ab on 2p1h;
// virtual q = o + a: -e_a.
__global__ void ea_rhs_kernel(const int64_t* __restrict__ orb, const double* __restrict__ t1,
                              const double* __restrict__ t2, double* __restrict__ out, int64_t o, int64_t v,
                              int64_t p1, int64_t Dp) {
  const int64_t r = blockIdx.y, q = orb[r];
  double* row = out + r * Dp;
  const int64_t n2 = o * v * v;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < Dp; t += int64_t(gridDim.x) * blockDim.x) {
    double val = 0.0;
    if (q < o) {
      if (t < v)
        val = t1[q * v + t];
      else if (t >= p1 && t - p1 < n2)
        val = t2[q * n2 + (t - p1)];
    } else if (t == q - o) {
      val = -1.0;
    }
    row[t] = val;
  }
}

// left vectors c'_p = <Phi|(1 + Lambda) abar_p on 1p + 2p1h, with ul[i,j,b,c] = 2 l2[i,j,b,c] - l2[i,j,c,b]:
//   occupied p = i:     1p[b] = -l1[i,b];   2p1h[j,b,c] = -ul[i,j,b,c]
//   virtual p = o + a:  1p[b] = d_ab - sum_i l1[i,b] t1[i,a] - Sl[a,b]
//                       2p1h[j,b,c] = 2 d_ab l1[j,c] - d_ac l1[j,b] - sum_i t1[i,a] ul[i,j,b,c]
__global__ void ea_left_kernel(const int64_t* __restrict__ orb, const double* __restrict__ t1,
                               const double* __restrict__ l1, const double* __restrict__ l2,
                               const double* __restrict__ Sl, double* __restrict__ out, int64_t o, int64_t v,
                               int64_t p1, int64_t Dp) {
  const int64_t r = blockIdx.y, p = orb[r];
  double* row = out + r * Dp;
  const int64_t vv = v * v, n2 = o * vv;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < Dp; t += int64_t(gridDim.x) * blockDim.x) {
    double val = 0.0;
    if (t < v) {
      const int64_t b = t;
      if (p < o) {
        val = -l1[p * v + b];
      } else {
        const int64_t a = p - o;
        val = (a == b ? 1.0 : 0.0) - Sl[a * v + b];
        for (int64_t i = 0; i < o; ++i) val -= l1[i * v + b] * t1[i * v + a];
      }
    } else if (t >= p1 && t - p1 < n2) {
      const int64_t idx = t - p1, j = idx / vv, b = (idx / v) % v, cc = idx % v;
      if (p < o) {
        const int64_t base = (p * o + j) * vv;
        val = -(2.0 * l2[base + b * v + cc] - l2[base + cc * v + b]);
      } else {
        const int64_t a = p - o;
        if (a == b) val += 2.0 * l1[j * v + cc];
        if (a == cc) val -= l1[j * v + b];
        for (int64_t i = 0; i < o; ++i) {
          const int64_t base = (i * o + j) * vv;
          val -= t1[i * v + a] * (2.0 * l2[base + b * v + cc] - l2[base + cc * v + b]);
        }
      }
    }
    row[t] = val;
  }
}

// FP64 product on the large double-buffered tile when it fills the GPU, else the default tile or split-K
void run64(gfcc_ctx* c, const GemmArgs& g, hipStream_t s) {
  if (!g.b_ncontig && g.batch == 1 && g.M >= 2048 && g.N >= 2048 && g.K >= 256)
    gemm(Prec::F64, g, gemm_big_cfg(Prec::F64, g.M, g.N, g.K), s);
  else
    gemm_auto(Prec::F64, g, c->scr, 3, s);
}

}  // namespace

// ------------------------------------------------------------------ build

void build_ea(gfcc_ctx* c, const gfcc_system* sys, hipStream_t s) {
  const int64_t o = c->o, v = c->v, Q = c->Q, n = c->n, ov = c->ov, kp = c->kp, p1 = c->p1, Dp = c->Dp;
  const int64_t vv = v * v, vp = c->vp;
  c->ea.lv = round_up(vv, 8);
  c->ea.n2p = round_up(o * vv, 8);
  const int64_t lv = c->ea.lv, n2p = c->ea.n2p;
  Scratch& scr = c->scr;
  auto g64 = [&](DBuf& b, int64_t nd) {
    b.ensure(size_t(nd) * 8, s);
    return b.as<double>();
  };
  double* Lp = const_cast<double*>(sys->L);
  const TView Lov = tview_s(Lp + o, {Q, o, v}, {n * n, n, 1});
  const TView Loo = tview_s(Lp, {Q, o, o}, {n * n, n, 1});
  const TView Lvv = tview_s(Lp + o * n + o, {Q, v, v}, {n * n, n, 1});

  // inputs kept by the context: t1, l1 copies; t2 (and l2) borrowed
  double* t1p = g64(c->t1c, o * v);
  GFCC_HIP(hipMemcpyAsync(t1p, sys->t1, size_t(o * v) * 8, hipMemcpyDeviceToDevice, s));
  double* l1p = g64(c->l1c, o * v);
  GFCC_HIP(hipMemcpyAsync(l1p, sys->l1 ? sys->l1 : sys->t1, size_t(o * v) * 8, hipMemcpyDeviceToDevice, s));
  c->t2 = sys->t2;
  c->l2 = (sys->l2 && sys->l2 != sys->t2) ? sys->l2 : nullptr;
  const TView t1 = tview(t1p, {o, v});
  const TView t2 = tview(const_cast<double*>(sys->t2), {o, o, v, v});

  // integral blocks and amplitude combinations (build temporaries)
  DBuf b_ovov, b_ooov, b_oovv, b_ovvv, b_M, b_ut, b_tau, b_Wvo, b_Wov, b_tmp, b_Y;
  const TView ovov = tview(g64(b_ovov, ov * ov), {o, v, o, v});
  const TView ooov = tview(g64(b_ooov, o * o * ov), {o, o, o, v});
  const TView oovv = tview(g64(b_oovv, o * o * vv), {o, o, v, v});
  const TView ovvv = tview(g64(b_ovvv, ov * vv), {o, v, v, v});
  ein("Qkc,Qld->kcld", 1.0, Lov, Lov, 0.0, ovov, scr, s);
  ein("Qmn,Qkc->mnkc", 1.0, Loo, Lov, 0.0, ooov, scr, s);
  ein("Qmn,Qab->mnab", 1.0, Loo, Lvv, 0.0, oovv, scr, s);
  ein("Qkc,Qab->kcab", 1.0, Lov, Lvv, 0.0, ovvv, scr, s);
  // T1-dressed Cholesky vectors M[Q,a,c] = L[Q,a,c] - sum_k t_ka L[Q,k,c]
  const TView M = tview(g64(b_M, Q * vv), {Q, v, v});
  {
    const int id[3] = {0, 1, 2};
    permute(Lvv, id, 1.0, M, 0.0, s);
  }
  ein("ka,Qkc->Qac", -1.0, t1, Lov, 1.0, M, scr, s);
  const TView ut = tview(g64(b_ut, o * o * vv), {o, o, v, v});
  const TView tau = tview(g64(b_tau, o * o * vv), {o, o, v, v});
  hipLaunchKernelGGL(unsym_kernel, dim3(nblk(o * o * vv)), dim3(256), 0, s, sys->t2, ut.p, o, v);
  hipLaunchKernelGGL(tau_kernel, dim3(nblk(o * o * vv)), dim3(256), 0, s, sys->t2, t1p, tau.p, o, v);
  GFCC_HIP(hipGetLastError());

  // one-body blocks (paper, Implementation Details: constant intermediates of Hbar)
  const TView Fov = tview(g64(c->Fov, ov), {o, v});
  const TView Foo = tview(g64(c->Foo, o * o), {o, o});
  const TView Fvv = tview(g64(c->Fvv, vv), {v, v});
  ein("nf,menf->me", 2.0, t1, ovov, 0.0, Fov, scr, s);
  ein("nf,mfne->me", -1.0, t1, ovov, 1.0, Fov, scr, s);
  GFCC_HIP(hipMemsetAsync(Foo.p, 0, size_t(o * o) * 8, s));
  GFCC_HIP(hipMemsetAsync(Fvv.p, 0, size_t(vv) * 8, s));
  hipLaunchKernelGGL(add_eps_kernel, dim3(nblk(o)), dim3(256), 0, s, Foo.p, sys->eps, o);
  hipLaunchKernelGGL(add_eps_kernel, dim3(nblk(v)), dim3(256), 0, s, Fvv.p, sys->eps + o, v);
  GFCC_HIP(hipGetLastError());
  ein("ie,me->mi", 1.0, t1, Fov, 1.0, Foo, scr, s);
  ein("ne,mine->mi", 2.0, t1, ooov, 1.0, Foo, scr, s);
  ein("ne,nime->mi", -1.0, t1, ooov, 1.0, Foo, scr, s);
  ein("inef,menf->mi", 1.0, ut, ovov, 1.0, Foo, scr, s);
  ein("ma,me->ae", -1.0, t1, Fov, 1.0, Fvv, scr, s);
  ein("mf,mfae->ae", 2.0, t1, ovvv, 1.0, Fvv, scr, s);
  ein("mf,meaf->ae", -1.0, t1, ovvv, 1.0, Fvv, scr, s);
  ein("mnaf,menf->ae", -1.0, ut, ovov, 1.0, Fvv, scr, s);

  // ring blocks Wovvo[m,a,e,j], Wovov[m,a,j,e]
  const TView Wvo = tview(g64(b_Wvo, ov * ov), {o, v, v, o});
  const TView Wov = tview(g64(b_Wov, ov * ov), {o, v, o, v});
  const TView tmp = tview(g64(b_tmp, o * o * ov), {o, o, o, v});  // o^3 v scratch, relabelled per use
  {
    const int p_vo[4] = {0, 3, 1, 2};  // (me|ja) -> [m,a,e,j]
    permute(ovov, p_vo, 1.0, Wvo, 0.0, s);
    const int p_ov[4] = {0, 2, 1, 3};  // (mj|ae) -> [m,a,j,e]
    permute(oovv, p_ov, 1.0, Wov, 0.0, s);
  }
  ein("jnaf,menf->maej", 1.0, ut, ovov, 1.0, Wvo, scr, s);
  ein("jnaf,mfne->maej", -1.0, t2, ovov, 1.0, Wvo, scr, s);
  ein("jf,meaf->maej", 1.0, t1, ovvv, 1.0, Wvo, scr, s);
  ein("na,njme->maej", -1.0, t1, ooov, 1.0, Wvo, scr, s);
  {
    const TView G = tview(tmp.p, {o, v, o, o});  // G[m,e,n,j] = sum_f (me|nf) t_jf
    ein("menf,jf->menj", 1.0, ovov, t1, 0.0, G, scr, s);
    ein("na,menj->maej", -1.0, t1, G, 1.0, Wvo, scr, s);
  }
  ein("jnfa,mfne->maje", -1.0, t2, ovov, 1.0, Wov, scr, s);
  ein("jf,mfae->maje", 1.0, t1, ovvv, 1.0, Wov, scr, s);
  ein("na,mjne->maje", -1.0, t1, ooov, 1.0, Wov, scr, s);
  {
    const TView H = tview(tmp.p, {o, o, o, v});  // H[m,j,n,e] = sum_f t_jf (mf|ne)
    ein("jf,mfne->mjne", 1.0, t1, ovov, 0.0, H, scr, s);
    ein("na,mjne->maje", -1.0, t1, H, 1.0, Wov, scr, s);
  }

  // ring matrices of the 2p1h <- 2p1h product, one-body terms folded in
  double* R = g64(c->ea.ring, ov * 2 * kp);
  double* R2 = g64(c->ea.ring2, ov * kp);
  {
    const TView r1 = tview_s(R, {o, v, o, v}, {v * 2 * kp, 2 * kp, v, 1});       // [j,b,l,d]
    const TView r1b = tview_s(R + kp, {o, v, o, v}, {v * 2 * kp, 2 * kp, v, 1});  // [j,b,l,c]
    const TView r2 = tview_s(R2, {o, v, o, v}, {v * kp, kp, v, 1});               // [j,a,l,c]
    const int p_vo[4] = {3, 1, 0, 2};  // Wovvo[l,b,d,j] -> [j,b,l,d]
    const int p_ov[4] = {2, 1, 0, 3};  // Wovov[l,b,j,d] -> [j,b,l,d]
    permute(Wvo, p_vo, 2.0, r1, 0.0, s);
    permute(Wov, p_ov, -1.0, r1, 1.0, s);
    permute(Wvo, p_vo, -1.0, r1b, 0.0, s);
    permute(Wov, p_ov, -1.0, r2, 0.0, s);
    hipLaunchKernelGGL(ring_fold_kernel, dim3(nblk(ov * ov)), dim3(256), 0, s, R, R2, Foo.p, Fvv.p, o, v, kp);
    GFCC_HIP(hipGetLastError());
  }

  // three-body operator zop[k][(l,c,d)] = 2 (kc|ld) - (kd|lc)
  double* Z = g64(c->ea.zop, o * n2p);
  {
    const TView zv = tview_s(Z, {o, o, v, v}, {n2p, vv, v, 1});  // [k,l,c,d]
    const int pa[4] = {0, 2, 1, 3};  // ovov[k,c,l,d] -> [k,l,c,d]
    const int pb[4] = {0, 2, 3, 1};  // ovov[k,d,l,c] -> [k,l,c,d]
    permute(ovov, pa, 2.0, zv, 0.0, s);
    permute(ovov, pb, -1.0, zv, 1.0, s);
  }

  // ladder Wvvvv[(a,b)][(c,d)] = sum_Q M[Q,a,c] M[Q,b,d] + sum_kl t_kl^ab (kc|ld)
  double* W = g64(c->ea.ladder, vv * lv);
  const TView lad = tview_s(W, {v, v, v, v}, {v * lv, lv, v, 1});
  ein("Qac,Qbd->abcd", 1.0, M, M, 0.0, lad, scr, s);
  ein("klab,kcld->abcd", 1.0, t2, ovov, 1.0, lad, scr, s);

  // 1p <- plane: Uop[a] = [Fvv[a,:] | 2 Wvovv[a,l,c,d] - Wvovv[a,l,d,c] + Fov terms]
  double* U = g64(c->Uop, v * Dp);
  {
    const TView u2 = tview_s(U + p1, {v, o, v, v}, {Dp, vv, v, 1});  // [a,l,c,d]
    ein("Qac,Qld->alcd", 2.0, M, Lov, 0.0, u2, scr, s);
    ein("Qad,Qlc->alcd", -1.0, M, Lov, 1.0, u2, scr, s);
    hipLaunchKernelGGL(uop_fold_kernel, dim3(nblk(o * vv), unsigned(v)), dim3(256), 0, s, U, Fvv.p, Fov.p, o, v, p1,
                       Dp);
    GFCC_HIP(hipGetLastError());
  }

  // 2p1h <- 1p: WvvvoT[(j,a,b)][c] = Wvvvo[a,b,c,j]
  double* V5 = g64(c->ea.vvvoT, o * vv * vp);
  {
    const TView w = tview_s(V5, {o, v, v, v}, {vv * vp, v * vp, vp, 1});  // [j,a,b,c]
    ein("Qac,Qjb->jabc", 1.0, M, Lov, 0.0, w, scr, s);       // (ac|bj) - sum_m t_ma (mc|jb)
    ein("mc,mjab->jabc", -1.0, Fov, t2, 1.0, w, scr, s);
    ein("jf,abcf->jabc", 1.0, t1, lad, 1.0, w, scr, s);
    ein("njmc,mnab->jabc", 1.0, ooov, tau, 1.0, w, scr, s);  // (mc|nj) tau_mn^ab
    ein("mcbf,mjaf->jabc", -1.0, ovvv, t2, 1.0, w, scr, s);
    ein("mcaf,mjfb->jabc", -1.0, ovvv, t2, 1.0, w, scr, s);
    ein("mfac,mjfb->jabc", 1.0, ovvv, ut, 1.0, w, scr, s);
    const TView Y = tview(g64(b_Y, ov * ov), {o, v, v, o});
    // -sum_m t_ma Yb[m,b,c,j],  Yb = sum_nf (mc|nf)(2 t_nj^fb - t_nj^bf) - (mf|nc) t_nj^fb
    ein("mcnf,njfb->mbcj", 1.0, ovov, ut, 0.0, Y, scr, s);
    ein("mfnc,njfb->mbcj", -1.0, ovov, t2, 1.0, Y, scr, s);
    ein("ma,mbcj->jabc", -1.0, t1, Y, 1.0, w, scr, s);
    // +sum_m t_mb Ya[m,a,c,j],  Ya = -(mj|ac) + sum_nf (mf|nc) t_nj^af
    const int p_a[4] = {0, 2, 3, 1};  // oovv[m,j,a,c] -> [m,a,c,j]
    permute(oovv, p_a, -1.0, Y, 0.0, s);
    ein("mfnc,njaf->macj", 1.0, ovov, t2, 1.0, Y, scr, s);
    ein("mb,macj->jabc", 1.0, t1, Y, 1.0, w, scr, s);
  }

  // left-vector helper Sl[a,b] = sum_ijc t2[i,j,a,c] (2 l2[i,j,b,c] - l2[i,j,c,b])
  {
    hipLaunchKernelGGL(unsym_kernel, dim3(nblk(o * o * vv)), dim3(256), 0, s, c->l2 ? c->l2 : sys->t2, ut.p, o, v);
    GFCC_HIP(hipGetLastError());
    const TView Sl = tview(g64(c->ea.Sl, vv), {v, v});
    ein("ijac,ijbc->ab", 1.0, t2, ut, 0.0, Sl, scr, s);
  }

  // exact diagonal
  double* dg = g64(c->diag, Dp);
  hipLaunchKernelGGL(ea_diag_kernel, dim3(nblk(Dp)), dim3(256), 0, s, dg, Fvv.p, W, R, R2, Z, sys->t2, o, v, p1, Dp,
                     kp, lv, n2p);
  GFCC_HIP(hipGetLastError());
  GFCC_HIP(hipStreamSynchronize(s));  // build temporaries are released on return
}

// ------------------------------------------------------------------ sigma

static void ea_sigma_f16(gfcc_ctx* c, int64_t P, const double* x, double* y, hipStream_t s);

void ea_sigma_planes(gfcc_ctx* c, int64_t P, const double* x, double* y, gfcc_precision prec, hipStream_t s) {
  if (P <= 0) return;
  if (prec == GFCC_FP16_IR) {
    ea_sigma_f16(c, P, x, y, s);
    return;
  }
  const int64_t o = c->o, v = c->v, ov = c->ov, kp = c->kp, p1 = c->p1, Dp = c->Dp, vv = v * v;
  const int64_t n2 = c->n2, lv = c->ea.lv, n2p = c->ea.n2p, op = round_up(o, 8);
  c->ea.ws_R.ensure(size_t(P * v * 2 * kp) * 8, s);
  c->ea.ws_z.ensure(size_t(P * op) * 8, s);
  double* R = c->ea.ws_R.as<double>();
  double* z = c->ea.ws_z.as<double>();
  prof_begin(c, "ea_sigma", s);

  // 1p <- plane
  {
    GemmArgs g;
    g.A = x; g.am = lin(Dp);
    g.B = c->Uop.as<double>(); g.bm = lin(Dp);
    g.C = y; g.cm = lin(Dp); g.cn = lin(1);
    g.M = P; g.N = v; g.K = Dp;
    run64(c, g, s);
  }
  // 2p1h <- 1p (initialises the 2p1h block)
  {
    GemmArgs g;
    g.A = x; g.am = lin(Dp);
    g.B = c->ea.vvvoT.as<double>(); g.bm = lin(c->vp);
    g.C = y + p1; g.cm = lin(Dp); g.cn = lin(1);
    g.M = P; g.N = n2; g.K = v;
    run64(c, g, s);
  }
  // ring products
  hipLaunchKernelGGL((ea_ring_operand_kernel<double>), dim3(unsigned(P * v)), dim3(256), 0, s, x, R, o, v, p1, Dp, kp,
                     nullptr);
  GFCC_HIP(hipGetLastError());
  {
    GemmArgs g;  // rows (x,a), cols (j,b): s2[x,j,a,b]
    g.A = R; g.am = lin(2 * kp);
    g.B = c->ea.ring.as<double>(); g.bm = lin(2 * kp);
    g.C = y + p1; g.cm = two(v, Dp, v); g.cn = two(v, vv, 1);
    g.M = P * v; g.N = ov; g.K = 2 * kp; g.beta = 1.0;
    prof_begin(c, "ea_ring", s);
    run64(c, g, s);
    prof_end(c, "ea_ring", s, 2.0 * double(g.M) * double(g.N) * double(g.K), 0.0);
  }
  {
    GemmArgs g;  // rows (x,b), cols (j,a): s2[x,j,a,b]
    g.A = R + kp; g.am = lin(2 * kp);
    g.B = c->ea.ring2.as<double>(); g.bm = lin(kp);
    g.C = y + p1; g.cm = two(v, Dp, 1); g.cn = two(v, vv, v);
    g.M = P * v; g.N = ov; g.K = kp; g.beta = 1.0;
    run64(c, g, s);
  }
  // particle-particle ladder
  {
    GemmArgs g;  // rows (x,j), cols (a,b)
    g.A = x + p1; g.am = two(o, Dp, vv);
    g.B = c->ea.ladder.as<double>(); g.bm = lin(lv);
    g.C = y + p1; g.cm = two(o, Dp, vv); g.cn = lin(1);
    g.M = P * o; g.N = vv; g.K = vv; g.beta = 1.0;
    prof_begin(c, "ea_ladder", s);
    run64(c, g, s);
    prof_end(c, "ea_ladder", s, 2.0 * double(g.M) * double(g.N) * double(g.K),
             8.0 * (double(vv) * double(vv) + 2.0 * double(g.M) * double(vv)));
  }
  // three-body term: z[x,k] = sum zop[k] . y2[x];  y2[x] -= sum_k z[x,k] t2[k]
  {
    GemmArgs g;
    g.A = x + p1; g.am = lin(Dp);
    g.B = c->ea.zop.as<double>(); g.bm = lin(n2p);
    g.C = z; g.cm = lin(op); g.cn = lin(1);
    g.M = P; g.N = o; g.K = n2;
    run64(c, g, s);
    GemmArgs h;
    h.A = z; h.am = lin(op);
    h.B = c->t2; h.bm = lin(n2); h.b_ncontig = 1;
    h.C = y + p1; h.cm = lin(Dp); h.cn = lin(1);
    h.M = P; h.N = n2; h.K = o; h.alpha = -1.0; h.beta = 1.0;
    run64(c, h, s);
  }
  hipLaunchKernelGGL(zero_pads_kernel, dim3(1, unsigned(P)), dim3(256), 0, s, y, c->n1, p1, n2, Dp);
  GFCC_HIP(hipGetLastError());
  prof_end(c, "ea_sigma", s, 0.0, 0.0);
}

// ------------------------------------------------------------------ FP16 form

void build_ea_lowprec(gfcc_ctx* c, hipStream_t s) {
  auto& H = c->ea.h;
  if (H.built) return;
  const int64_t o = c->o, v = c->v, ov = c->ov, kp = c->kp, Dp = c->Dp, vv = v * v;
  auto mk = [&](DBuf& dst, const double* src, int64_t n, double& scale) {
    const double am = amax_host(src, n, s, c->scr);
    scale = (am > 0.0) ? std::ldexp(1.0, -std::ilogb(am)) : 1.0;  // amax -> [1, 2)
    dst.ensure(size_t(n) * 2, s);
    convert_f64(src, dst.p, Prec::F16, n, scale, s);
  };
  mk(H.ladder, c->ea.ladder.as<double>(), vv * c->ea.lv, H.sL);
  mk(H.vvvoT, c->ea.vvvoT.as<double>(), o * vv * c->vp, H.sV);
  mk(H.Uop, c->Uop.as<double>(), v * Dp, H.sU);
  mk(H.ring, c->ea.ring.as<double>(), ov * 2 * kp, H.sR);
  mk(H.ring2, c->ea.ring2.as<double>(), ov * kp, H.sR2);
  mk(H.zop, c->ea.zop.as<double>(), o * c->ea.n2p, H.sZ);
  mk(H.t2, c->t2, o * o * vv, H.sT);
  GFCC_HIP(hipStreamSynchronize(s));
  H.built = true;
}

// FP16 products with FP32 accumulation: the plane operands are scaled on the GPU (sc[0]) and every
// product undoes that scale from device memory; the three-body vector z gets a scale of its own.
static void ea_sigma_f16(gfcc_ctx* c, int64_t P, const double* x, double* y, hipStream_t s) {
  const int64_t o = c->o, v = c->v, ov = c->ov, kp = c->kp, p1 = c->p1, Dp = c->Dp, vv = v * v;
  const int64_t n2 = c->n2, lv = c->ea.lv, n2p = c->ea.n2p, op = round_up(o, 8);
  build_ea_lowprec(c, s);
  const auto& H = c->ea.h;
  c->ea.ws_xh.ensure(size_t(P * Dp) * 2, s);
  c->ea.ws_Rh.ensure(size_t(P * v * 2 * kp) * 2, s);
  c->ea.ws_z.ensure(size_t(P * op) * 8, s);
  c->ea.ws_zh.ensure(size_t(P * op) * 2, s);
  _Float16* xh = c->ea.ws_xh.as<_Float16>();
  _Float16* Rh = c->ea.ws_Rh.as<_Float16>();
  double* z = c->ea.ws_z.as<double>();
  _Float16* zh = c->ea.ws_zh.as<_Float16>();
  prof_begin(c, "ea_sigma", s);
  vector_scale(c, x, P * Dp, 0, s);
  const double* sc = c->ws_vsc.as<double>();
  hipLaunchKernelGGL(to_f16_scaled_kernel, dim3(nblk(P * Dp)), dim3(256), 0, s, x, xh, P * Dp, sc);
  hipLaunchKernelGGL((ea_ring_operand_kernel<_Float16>), dim3(unsigned(P * v)), dim3(256), 0, s, x, Rh, o, v, p1, Dp,
                     kp, sc);
  GFCC_HIP(hipGetLastError());
  auto run16 = [&](const GemmArgs& g) {
    if (!g.b_ncontig && g.batch == 1 && g.M >= 2048 && g.N >= 2048 && g.K >= 256)
      gemm(Prec::F16, g, gemm_big_cfg(Prec::F16, g.M, g.N, g.K), s);
    else
      gemm_auto(Prec::F16, g, c->scr, 3, s);
  };
  {  // 1p <- plane
    GemmArgs g;
    g.A = xh; g.am = lin(Dp);
    g.B = H.Uop.p; g.bm = lin(Dp);
    g.C = y; g.cm = lin(Dp); g.cn = lin(1);
    g.M = P; g.N = v; g.K = Dp;
    g.alpha = 1.0 / H.sU; g.alpha_dev = sc + 1;
    run16(g);
  }
  {  // 2p1h <- 1p
    GemmArgs g;
    g.A = xh; g.am = lin(Dp);
    g.B = H.vvvoT.p; g.bm = lin(c->vp);
    g.C = y + p1; g.cm = lin(Dp); g.cn = lin(1);
    g.M = P; g.N = n2; g.K = v;
    g.alpha = 1.0 / H.sV; g.alpha_dev = sc + 1;
    run16(g);
  }
  {
    GemmArgs g;  // ring 1: rows (x,a), cols (j,b)
    g.A = Rh; g.am = lin(2 * kp);
    g.B = H.ring.p; g.bm = lin(2 * kp);
    g.C = y + p1; g.cm = two(v, Dp, v); g.cn = two(v, vv, 1);
    g.M = P * v; g.N = ov; g.K = 2 * kp; g.beta = 1.0;
    g.alpha = 1.0 / H.sR; g.alpha_dev = sc + 1;
    prof_begin(c, "ea_ring", s);
    run16(g);
    prof_end(c, "ea_ring", s, 2.0 * double(g.M) * double(g.N) * double(g.K), 0.0);
  }
  {
    GemmArgs g;  // ring 2: rows (x,b), cols (j,a)
    g.A = Rh + kp; g.am = lin(2 * kp);
    g.B = H.ring2.p; g.bm = lin(kp);
    g.C = y + p1; g.cm = two(v, Dp, 1); g.cn = two(v, vv, v);
    g.M = P * v; g.N = ov; g.K = kp; g.beta = 1.0;
    g.alpha = 1.0 / H.sR2; g.alpha_dev = sc + 1;
    run16(g);
  }
  {
    GemmArgs g;  // ladder
    g.A = xh + p1; g.am = two(o, Dp, vv);
    g.B = H.ladder.p; g.bm = lin(lv);
    g.C = y + p1; g.cm = two(o, Dp, vv); g.cn = lin(1);
    g.M = P * o; g.N = vv; g.K = vv; g.beta = 1.0;
    g.alpha = 1.0 / H.sL; g.alpha_dev = sc + 1;
    prof_begin(c, "ea_ladder", s);
    run16(g);
    prof_end(c, "ea_ladder", s, 2.0 * double(g.M) * double(g.N) * double(g.K),
             2.0 * (double(vv) * double(vv) + 2.0 * double(g.M) * double(vv)));
  }
  {  // three-body: z (carrying sc[0]) = y2 . zop, then y2 -= z . t2 with z scaled by sc[2]
    // (the pad columns of z enter its scale, so they are cleared first)
    hipLaunchKernelGGL(fill_zero_kernel, dim3(nblk(P * op)), dim3(256), 0, s, z, P * op);
    GemmArgs g;
    g.A = xh + p1; g.am = lin(Dp);
    g.B = H.zop.p; g.bm = lin(n2p);
    g.C = z; g.cm = lin(op); g.cn = lin(1);
    g.M = P; g.N = o; g.K = n2;
    g.alpha = 1.0 / H.sZ;
    run16(g);
    vector_scale(c, z, P * op, 1, s);
    hipLaunchKernelGGL(to_f16_scaled_kernel, dim3(nblk(P * op)), dim3(256), 0, s, z, zh, P * op, sc + 2);
    GFCC_HIP(hipGetLastError());
    GemmArgs h;
    h.A = zh; h.am = lin(op);
    h.B = H.t2.p; h.bm = lin(n2); h.b_ncontig = 1;
    h.C = y + p1; h.cm = lin(Dp); h.cn = lin(1);
    h.M = P; h.N = n2; h.K = o; h.beta = 1.0;
    h.alpha = -1.0 / H.sT; h.alpha_dev = sc + 3;
    run16(h);
  }
  hipLaunchKernelGGL(zero_pads_kernel, dim3(1, unsigned(P)), dim3(256), 0, s, y, c->n1, p1, n2, Dp);
  GFCC_HIP(hipGetLastError());
  prof_end(c, "ea_sigma", s, 0.0, 0.0);
}

void ea_rhs_rows(gfcc_ctx* c, int64_t n, const int64_t* orb_dev, double* out, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(ea_rhs_kernel, dim3(nblk(c->Dp), unsigned(n)), dim3(256), 0, s, orb_dev, c->t1c.as<double>(),
                     c->t2, out, c->o, c->v, c->p1, c->Dp);
  GFCC_HIP(hipGetLastError());
}

void ea_left_rows(gfcc_ctx* c, int64_t n, const int64_t* orb_dev, double* out, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(ea_left_kernel, dim3(nblk(c->Dp), unsigned(n)), dim3(256), 0, s, orb_dev, c->t1c.as<double>(),
                     c->l1c.as<double>(), c->l2 ? c->l2 : c->t2, c->ea.Sl.as<double>(), out, c->o, c->v, c->p1,
                     c->Dp);
  GFCC_HIP(hipGetLastError());
}

}  // namespace gfcc

// Per-system intermediates of the IP-GFCCSD sigma product, built on the GPU.
//
// The paper precomputes constant intermediates of size <= O(o^2 v^2) before
// the GFCC loop (Implementation Details) and evaluates the GFCCSD equations (Theory, T and
// Lambda at the two-body level, X_p in the 1h + 2h1p space) as tensor
// contractions of T1/T2 with Cholesky-decomposed integrals.  The closed-shell
// spin-adapted blocks of the connected Hbar_N built here are
//   Fov[m,e]  = sum_nf t_nf [2(me|nf) - (mf|ne)]
//   Foo[m,i]  = e_i d_mi + sum_e t_ie Fov[m,e] + sum_ne t_ne [2(mi|ne) - (me|ni)]
//               + sum_nef (2 t_in^ef - t_in^fe)(me|nf)
//   Fvv[a,e]  = e_a d_ae - sum_m t_ma Fov[m,e] + sum_mf t_mf [2(ae|mf) - (af|me)]
//               - sum_mnf (2 t_mn^af - t_mn^fa)(me|nf)
//   Woooo[m,n,i,j] = (mi|nj) + sum_e [t_je (mi|ne) + t_ie (me|nj)] + sum_ef tau_ij^ef (me|nf)
//   Wooov[m,n,i,e] = (mi|ne) + sum_f t_if (mf|ne)
//   Qovvo[m,a,e,j] = (me|aj) + sum_nf [(2 t_jn^af - t_jn^fa)(me|nf) - t_jn^af (mf|ne)]
//   Qovov[m,a,j,e] = (mj|ae) - sum_nf t_jn^fa (mf|ne)
//   Wovvo = Qovvo + sum_f t_jf (me|af) - sum_n t_na (me|nj) - sum_nf t_jf t_na (me|nf)
//   Wovov = Qovov + sum_f t_jf (mf|ae) - sum_n t_na (mj|ne) - sum_nf t_jf t_na (mf|ne)
//   Wovoo[m,a,i,j] = (mi|aj) + sum_e Fov[m,e] t_ij^ea - sum_n t_na Woooo[m,n,i,j]
//               + sum_ef (me|af) tau_ij^ef + sum_ne [(mi|ne)(2 t_jn^ae - t_jn^ea)
//               - (me|ni) t_jn^ae - (me|nj) t_in^ea] + sum_e [t_ie Qovvo[m,a,e,j] + t_je Qovov[m,a,i,e]]
// with (pq|rs) = sum_Q L[Q,p,q] L[Q,r,s] and tau_ij^ef = t_ij^ef + t_ie t_jf.
// Integrals with three virtual indices are never stored whole: they are
// contracted through L (t1 terms) or formed in occupied-index chunks (tau term).
#include <algorithm>
#include <cmath>

#include "ctx.h"

namespace gfcc {

__global__ void add_diag_kernel(double* p, int64_t n, int64_t stride, const double* src, double alpha,
                                double beta) {
  int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < n) p[t * stride] = beta * p[t * stride] + alpha * (src ? src[t] : 1.0);
}

static void add_diag(double* p, int64_t n, int64_t stride, const double* src, double alpha, double beta,
                     hipStream_t s) {
  hipLaunchKernelGGL(add_diag_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, p, n, stride, src,
                     alpha, beta);
  GFCC_HIP(hipGetLastError());
}

// Exact diagonal of Hbar_N over the plane layout.
// flag = 1 when a[0:n] and b[0:n] differ anywhere
__global__ void differ_kernel(const double* __restrict__ a, const double* __restrict__ b, int64_t n, int* flag) {
  bool d = false;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n; t += int64_t(gridDim.x) * blockDim.x)
    d = d || (a[t] != b[t]);
  if (d) *flag = 1;
}

__global__ void diag_kernel(double* __restrict__ dg, int64_t o, int64_t v, int64_t o_pad, int64_t kp,
                            const double* __restrict__ Foo, const double* __restrict__ Fvv,
                            const double* __restrict__ Woooo, const double* __restrict__ Wvo,
                            const double* __restrict__ Wov, const double* __restrict__ ovov,
                            const double* __restrict__ t2) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t oov = o * o * v;
  if (t < o) dg[t] = -Foo[t * o + t];
  if (t >= oov) return;
  const int64_t a = t % v, j = (t / v) % o, i = t / (o * v);
  const int64_t ov = o * v;
  auto wvo = [&](int64_t m, int64_t aa, int64_t e, int64_t jj) { return Wvo[(jj * v + aa) * kp + m * v + e]; };
  auto wov = [&](int64_t m, int64_t aa, int64_t jj, int64_t e) { return Wov[(jj * v + aa) * kp + m * v + e]; };
  double d = Fvv[a * v + a] - Foo[i * o + i] - Foo[j * o + j];
  d += Woooo[((i * o + j) * o + i) * o + j];
  d += 2.0 * wvo(j, a, a, j) - wov(j, a, j, a);
  if (i == j) d -= wvo(i, a, a, i);
  d -= wov(i, a, i, a);
  double tb = 0.0;
  for (int64_t e = 0; e < v; ++e) {
    const double g1 = ovov[((i * v + e) * o + j) * v + a];  // (ie|ja)
    const double g2 = ovov[((i * v + a) * o + j) * v + e];  // (ia|je)
    tb += (2.0 * g1 - g2) * t2[((i * o + j) * v + e) * v + a];
  }
  (void)ov;
  dg[o_pad + t] = d - tb;
}

void build_intermediates(gfcc_ctx* c, const gfcc_system* sys, hipStream_t s) {
  const int64_t o = c->o, v = c->v, Q = c->Q, n = c->n;
  const int64_t ov = o * v, oo = o * o, oov = oo * v, ovv = ov * v, n_oovv = oo * v * v;
  Scratch& scr = c->scr;
  double* L = const_cast<double*>(sys->L);
  double* t1 = const_cast<double*>(sys->t1);
  double* t2 = const_cast<double*>(sys->t2);
  double* l1 = const_cast<double*>(sys->l1 ? sys->l1 : sys->t1);
  double* l2 = const_cast<double*>(sys->l2 ? sys->l2 : sys->t2);

  const double* eps = sys->eps;

  const int64_t nn = n * n;
  TView Loo = tview_s(L, {Q, o, o}, {nn, n, 1});
  TView Lov = tview_s(L + o, {Q, o, v}, {nn, n, 1});
  TView Lvv = tview_s(L + o * n + o, {Q, v, v}, {nn, n, 1});
  TView T1 = tview(t1, {o, v});
  TView T2 = tview(t2, {o, o, v, v});

  // ---- integral blocks
  DBuf b_ovov, b_oovv, b_ooov, b_oooo, b_tau, b_u2;
  b_ovov.ensure(n_oovv * 8, s);
  b_oovv.ensure(n_oovv * 8, s);
  b_ooov.ensure(oov * o * 8, s);
  b_oooo.ensure(oo * oo * 8, s);
  TView ovov = tview(b_ovov.as<double>(), {o, v, o, v});   // (me|nf)
  TView oovv = tview(b_oovv.as<double>(), {o, o, v, v});   // (mi|ae)
  TView ooov = tview(b_ooov.as<double>(), {o, o, o, v});   // (mi|ne)
  TView oooo = tview(b_oooo.as<double>(), {o, o, o, o});   // (mi|nj)
  ein("Qme,Qnf->menf", 1.0, Lov, Lov, 0.0, ovov, scr, s);
  ein("Qmi,Qae->miae", 1.0, Loo, Lvv, 0.0, oovv, scr, s);
  ein("Qmi,Qne->mine", 1.0, Loo, Lov, 0.0, ooov, scr, s);
  ein("Qmi,Qnj->minj", 1.0, Loo, Loo, 0.0, oooo, scr, s);

  // tau = t2 + t1 t1 ; u2 = 2 t2 - t2^(ab swapped)
  b_tau.ensure(n_oovv * 8, s);
  b_u2.ensure(n_oovv * 8, s);
  TView tau = tview(b_tau.as<double>(), {o, o, v, v});
  TView u2 = tview(b_u2.as<double>(), {o, o, v, v});
  GFCC_HIP(hipMemcpyAsync(tau.p, t2, n_oovv * 8, hipMemcpyDeviceToDevice, s));
  ein("ie,jf->ijef", 1.0, T1, T1, 1.0, tau, scr, s);
  {
    const int id[4] = {0, 1, 2, 3}, sw[4] = {0, 1, 3, 2};
    permute(T2, id, 2.0, u2, 0.0, s);
    permute(T2, sw, -1.0, u2, 1.0, s);
  }

  // ---- one-body blocks
  c->Fov.ensure(ov * 8, s);
  c->Foo.ensure(oo * 8, s);
  c->Fvv.ensure(v * v * 8, s);
  TView Fov = tview(c->Fov.as<double>(), {o, v});
  TView Foo = tview(c->Foo.as<double>(), {o, o});
  TView Fvv = tview(c->Fvv.as<double>(), {v, v});
  ein("nf,menf->me", 2.0, T1, ovov, 0.0, Fov, scr, s);
  ein("nf,mfne->me", -1.0, T1, ovov, 1.0, Fov, scr, s);

  add_diag(Foo.p, o, o + 1, eps, 1.0, 0.0, s);
  ein("ie,me->mi", 1.0, T1, Fov, 1.0, Foo, scr, s);
  ein("ne,mine->mi", 2.0, T1, ooov, 1.0, Foo, scr, s);
  ein("ne,nime->mi", -1.0, T1, ooov, 1.0, Foo, scr, s);
  ein("inef,menf->mi", 1.0, u2, ovov, 1.0, Foo, scr, s);

  DBuf b_xq, b_Y, b_P;
  b_xq.ensure(Q * 8, s);
  b_Y.ensure(Q * v * o * 8, s);
  b_P.ensure(Q * o * o * 8, s);
  TView xQ = tview(b_xq.as<double>(), {Q});
  TView Y = tview(b_Y.as<double>(), {Q, v, o});   // Y[Q,a,j] = sum_f L[Q,a,f] t_jf
  TView P = tview(b_P.as<double>(), {Q, o, o});   // P[Q,m,j] = sum_f L[Q,m,f] t_jf
  ein("mf,Qmf->Q", 1.0, T1, Lov, 0.0, xQ, scr, s);
  ein("Qaf,jf->Qaj", 1.0, Lvv, T1, 0.0, Y, scr, s);
  ein("Qmf,jf->Qmj", 1.0, Lov, T1, 0.0, P, scr, s);

  add_diag(Fvv.p, v, v + 1, eps + o, 1.0, 0.0, s);
  ein("ma,me->ae", -1.0, T1, Fov, 1.0, Fvv, scr, s);
  ein("Q,Qae->ae", 2.0, xQ, Lvv, 1.0, Fvv, scr, s);          // 2 sum_mf t_mf (mf|ae)
  ein("Qme,Qam->ae", -1.0, Lov, Y, 1.0, Fvv, scr, s);        // - sum_mf t_mf (me|af)
  ein("mnaf,menf->ae", -1.0, u2, ovov, 1.0, Fvv, scr, s);

  // ---- Woooo, Wooov
  c->Woooo.ensure(oo * oo * 8, s);
  c->Wooov.ensure(oov * o * 8, s);
  TView Woooo = tview(c->Woooo.as<double>(), {o, o, o, o});
  TView Wooov = tview(c->Wooov.as<double>(), {o, o, o, v});
  {
    const int p4[4] = {0, 2, 1, 3};  // (mi|nj) -> [m][n][i][j];  (mi|ne) -> [m][n][i][e]
    permute(oooo, p4, 1.0, Woooo, 0.0, s);
    permute(ooov, p4, 1.0, Wooov, 0.0, s);
  }
  ein("je,mine->mnij", 1.0, T1, ooov, 1.0, Woooo, scr, s);
  ein("ie,njme->mnij", 1.0, T1, ooov, 1.0, Woooo, scr, s);
  ein("ijef,menf->mnij", 1.0, tau, ovov, 1.0, Woooo, scr, s);
  ein("if,mfne->mnie", 1.0, T1, ovov, 1.0, Wooov, scr, s);

  // ---- ring blocks, stored as [(j,a)][(m,e)] rows of length kp
  const int64_t kp = c->kp;
  c->Wvo.ensure(ov * kp * 8, s);
  c->Wov.ensure(ov * kp * 8, s);
  c->X1.ensure(ov * kp * 8, s);
  // view "jame" over [(j,a)][(m,e)]
  TView Wvo_jame = tview_s(c->Wvo.as<double>(), {o, v, o, v}, {v * kp, kp, v, 1});
  TView Wov_jame = tview_s(c->Wov.as<double>(), {o, v, o, v}, {v * kp, kp, v, 1});
  // the same storage seen as Wovvo[m,a,e,j] and Wovov[m,a,j,e]
  TView Wovvo = tview_s(c->Wvo.as<double>(), {o, v, v, o}, {v, kp, 1, v * kp});
  TView Wovov = tview_s(c->Wov.as<double>(), {o, v, o, v}, {v, kp, v * kp, 1});
  {
    const int pvo[4] = {0, 3, 1, 2};  // (me|aj) = ovov[m,e,j,a] -> Wovvo[m,a,e,j]
    permute(ovov, pvo, 1.0, Wovvo, 0.0, s);
    const int pov[4] = {0, 2, 1, 3};  // (mj|ae) = oovv[m,j,a,e] -> Wovov[m,a,j,e]
    permute(oovv, pov, 1.0, Wovov, 0.0, s);
  }
  ein("jnaf,menf->jame", 1.0, u2, ovov, 1.0, Wvo_jame, scr, s);
  ein("jnaf,mfne->jame", -1.0, T2, ovov, 1.0, Wvo_jame, scr, s);
  ein("jnfa,mfne->jame", -1.0, T2, ovov, 1.0, Wov_jame, scr, s);
  // (Wvo, Wov now hold Qovvo, Qovov)

  // ---- Wovoo (needs Qovvo, Qovov before their t1 terms are added)
  c->Wovoo.ensure(oov * o * 8, s);
  TView Wovoo = tview(c->Wovoo.as<double>(), {o, v, o, o});
  {
    const int p[4] = {0, 3, 1, 2};  // (mi|aj) = ooov[m,i,j,a] -> [m][a][i][j]
    permute(ooov, p, 1.0, Wovoo, 0.0, s);
  }
  ein("me,ijea->maij", 1.0, Fov, T2, 1.0, Wovoo, scr, s);
  ein("na,mnij->maij", -1.0, T1, Woooo, 1.0, Wovoo, scr, s);
  ein("mine,jnae->maij", 1.0, ooov, u2, 1.0, Wovoo, scr, s);
  ein("nime,jnae->maij", -1.0, ooov, T2, 1.0, Wovoo, scr, s);
  ein("njme,inea->maij", -1.0, ooov, T2, 1.0, Wovoo, scr, s);
  ein("ie,maej->maij", 1.0, T1, Wovvo, 1.0, Wovoo, scr, s);
  {
    TView Wovov_maie = Wovov;  // labels m,a,i,e over the same storage
    ein("je,maie->maij", 1.0, T1, Wovov_maie, 1.0, Wovoo, scr, s);
  }
  // sum_ef (me|af) tau_ij^ef in chunks of m: (me|af) = sum_Q L[Q,m,e] L[Q,a,f]
  {
    const int64_t bytes_per_m = v * v * v * 8;
    int64_t mc = std::max<int64_t>(1, std::min<int64_t>(o, (int64_t(1) << 30) / std::max<int64_t>(bytes_per_m, 1)));
    DBuf b_g;
    b_g.ensure(mc * v * v * v * 8, s);
    for (int64_t m0 = 0; m0 < o; m0 += mc) {
      const int64_t m1 = std::min(o, m0 + mc), cm = m1 - m0;
      TView Lc = tview_s(L + m0 * n + o, {Q, cm, v}, {nn, n, 1});
      TView G = tview(b_g.as<double>(), {cm, v, v, v});  // (me|af) for m in chunk
      ein("Qme,Qaf->meaf", 1.0, Lc, Lvv, 0.0, G, scr, s);
      TView Wc = tview_s(c->Wovoo.as<double>() + m0 * v * oo, {cm, v, o, o}, {v * oo, oo, o, 1});
      ein("meaf,ijef->maij", 1.0, G, tau, 1.0, Wc, scr, s);
    }
    GFCC_HIP(hipStreamSynchronize(s));  // b_g is freed at scope exit
  }

  // ---- t1 terms of the ring blocks
  {
    DBuf b_S;
    b_S.ensure(n_oovv * 8, s);
    TView S = tview(b_S.as<double>(), {o, v, o, o});  // S[m,e,n,j]
    ein("Qme,Qaj->jame", 1.0, Lov, Y, 1.0, Wvo_jame, scr, s);     // sum_f t_jf (me|af)
    ein("na,njme->jame", -1.0, T1, ooov, 1.0, Wvo_jame, scr, s);  // - sum_n t_na (me|nj)
    ein("menf,jf->menj", 1.0, ovov, T1, 0.0, S, scr, s);          // sum_f t_jf (me|nf)
    ein("na,menj->jame", -1.0, T1, S, 1.0, Wvo_jame, scr, s);
    ein("Qmj,Qae->jame", 1.0, P, Lvv, 1.0, Wov_jame, scr, s);     // sum_f t_jf (mf|ae)
    ein("na,mjne->jame", -1.0, T1, ooov, 1.0, Wov_jame, scr, s);  // - sum_n t_na (mj|ne)
    ein("mfne,jf->menj", 1.0, ovov, T1, 0.0, S, scr, s);          // sum_f t_jf (mf|ne)
    ein("na,menj->jame", -1.0, T1, S, 1.0, Wov_jame, scr, s);
    GFCC_HIP(hipStreamSynchronize(s));  // b_S is freed at scope exit
  }
  // X1 = 2 Wvo - Wov (padding stays zero)
  {
    TView a = tview(c->Wvo.as<double>(), {ov * kp});
    TView b = tview(c->Wov.as<double>(), {ov * kp});
    TView x = tview(c->X1.as<double>(), {ov * kp});
    const int id[1] = {0};
    permute(a, id, 2.0, x, 0.0, s);
    permute(b, id, -1.0, x, 1.0, s);
  }
  // Fold the off-diagonal one-body terms into the ring operands (exact):
  //   sum_e Fvv_off[a,e] r[i][j][e]   = sum_(m,e) d_jm Fvv_off[a,e] r[i][m][e]   -> X1 (P1a)
  //  -sum_m Foo_off[m,j] r[i][m][a]   = sum_(m,e) -d_ae Foo_off[m,j] r[i][m][e]  -> X1 (P1a)
  //  -sum_m Foo_off[m,i] r[m][j][a]   = -sum_(m,e) d_ae Foo_off[m,i] RT[j][m][e] -> Wov (P2, alpha -1)
  // The diagonal one-body part (Fvv[a,a] - Foo[i,i] - Foo[j,j]) r[i][j][a] is applied
  // elementwise in FP64 by the sigma operand kernel.
  {
    double* X1p = c->X1.as<double>();
    double* Wovp = c->Wov.as<double>();
    const int id3[3] = {0, 1, 2}, id2[2] = {0, 1};
    TView fvv_b = tview_s(c->Fvv.as<double>(), {o, v, v}, {0, v, 1});
    TView fvv_d = tview_s(c->Fvv.as<double>(), {o, v}, {0, v + 1});
    TView x_jm = tview_s(X1p, {o, v, v}, {v * kp + v, kp, 1});  // [j][a][e], m = j
    TView x_jd = tview_s(X1p, {o, v}, {v * kp + v, kp + 1});    // [j][a],    m = j, e = a
    permute(fvv_b, id3, 1.0, x_jm, 1.0, s);
    permute(fvv_d, id2, -1.0, x_jd, 1.0, s);
    TView foo_b = tview_s(c->Foo.as<double>(), {o, v, o}, {1, 0, o});  // [j][a][m] -> Foo[m][j]
    TView foo_d = tview_s(c->Foo.as<double>(), {o, v}, {o + 1, 0});    // [j][a]    -> Foo[j][j]
    TView x_ae = tview_s(X1p, {o, v, o}, {v * kp, kp + 1, v});        // [j][a][m], e = a
    permute(foo_b, id3, -1.0, x_ae, 1.0, s);
    permute(foo_d, id2, 1.0, x_jd, 1.0, s);
    TView w_ae = tview_s(Wovp, {o, v, o}, {v * kp, kp + 1, v});       // [i][a][m], e = a
    TView w_id = tview_s(Wovp, {o, v}, {v * kp + v, kp + 1});          // [i][a],    m = i, e = a
    permute(foo_b, id3, 1.0, w_ae, 1.0, s);
    permute(foo_d, id2, -1.0, w_id, 1.0, s);
  }
  // diagonal one-body part over the 2h1p block: d1b[(i,j,a)] = Fvv[a,a] - Foo[i,i] - Foo[j,j]
  c->d1b.ensure(oov * 8, s);
  {
    TView out = tview(c->d1b.as<double>(), {o, o, v});
    const int id3[3] = {0, 1, 2};
    permute(tview_s(c->Fvv.as<double>(), {o, o, v}, {0, 0, v + 1}), id3, 1.0, out, 0.0, s);
    permute(tview_s(c->Foo.as<double>(), {o, o, v}, {o + 1, 0, 0}), id3, -1.0, out, 1.0, s);
    permute(tview_s(c->Foo.as<double>(), {o, o, v}, {0, o + 1, 0}), id3, -1.0, out, 1.0, s);
  }

  // ---- sigma operands
  c->W4T.ensure(oo * c->op2 * 8, s);
  {
    TView w4t = tview_s(c->W4T.as<double>(), {o, o, o, o}, {o * c->op2, c->op2, o, 1});  // [i][j][m][n]
    const int p[4] = {2, 3, 0, 1};
    permute(Woooo, p, 1.0, w4t, 0.0, s);
  }
  c->Zm.ensure(v * c->ldz * 8, s);
  {
    TView z = tview_s(c->Zm.as<double>(), {v, o, o, v}, {c->ldz, ov, v, 1});  // [e][m][n][f]
    const int p1[4] = {1, 0, 2, 3};  // (me|nf): in dims (m,e,n,f)
    permute(ovov, p1, 2.0, z, 0.0, s);
    const int p2[4] = {3, 0, 2, 1};  // (mf|ne): in dims (m,f,n,e)
    permute(ovov, p2, -1.0, z, 1.0, s);
  }
  c->ktw = c->vp + c->o_pad;
  const int64_t ktw = c->ktw;
  c->TW.ensure(oov * ktw * 8, s);
  {
    TView t = tview_s(c->TW.as<double>(), {o, o, v, v}, {o * v * ktw, v * ktw, ktw, 1});  // [i][j][a][e]
    const int p[4] = {0, 1, 3, 2};
    permute(T2, p, 1.0, t, 0.0, s);
    TView w = tview_s(c->TW.as<double>() + c->vp, {o, o, v, o}, {o * v * ktw, v * ktw, ktw, 1});  // [i][j][a][m]
    const int q[4] = {2, 3, 1, 0};
    permute(Wovoo, q, 1.0, w, 0.0, s);
  }
  c->FooT.ensure(o * c->o_pad * 8, s);
  {
    TView f = tview_s(c->FooT.as<double>(), {o, o}, {c->o_pad, 1});
    const int tr[2] = {1, 0};
    permute(Foo, tr, 1.0, f, 0.0, s);
  }
  c->FvvM.ensure(v * c->vp * 8, s);
  {
    TView f = tview_s(c->FvvM.as<double>(), {v, v}, {c->vp, 1});
    const int id[2] = {0, 1};
    permute(Fvv, id, 1.0, f, 0.0, s);
  }
  // 1h rows: sigma_i = -sum_m Foo[m,i] r_m + sum_(mne) U[i,(m,n,e)] r_mne with
  // U = 2 d_im Fov[n,e] - d_in Fov[m,e] - 2 Wooov[m,n,i,e] + Wooov[n,m,i,e]
  const int64_t Dp = c->Dp, op = c->o_pad;
  c->Uop.ensure(o * Dp * 8, s);
  {
    double* U = c->Uop.as<double>();
    TView u1 = tview_s(U, {o, o}, {Dp, 1});  // [i][m]
    const int t2d[2] = {1, 0};
    permute(Foo, t2d, -1.0, u1, 0.0, s);
    TView u2v = tview_s(U + op, {o, o, o, v}, {Dp, ov, v, 1});  // [i][m][n][e]
    const int pa[4] = {2, 0, 1, 3}, pb[4] = {2, 1, 0, 3};
    permute(Wooov, pa, -2.0, u2v, 0.0, s);
    permute(Wooov, pb, 1.0, u2v, 1.0, s);
    TView fb = tview_s(c->Fov.as<double>(), {o, o, v}, {0, v, 1});  // broadcast over i
    const int id3[3] = {0, 1, 2};
    TView dq = tview_s(U + op, {o, o, v}, {Dp + ov, v, 1});  // i = m:  [i][n][e]
    permute(fb, id3, 2.0, dq, 1.0, s);
    TView dn = tview_s(U + op, {o, o, v}, {Dp + v, ov, 1});  // i = n:  [i][m][e]
    permute(fb, id3, -1.0, dn, 1.0, s);
  }

  // ---- exact diagonal (padding set to 1 so that Jacobi keeps zeros)
  c->diag.ensure(Dp * 8, s);
  {
    std::vector<double> ones(size_t(Dp), 1.0);
    GFCC_HIP(hipMemcpyAsync(c->diag.p, ones.data(), Dp * 8, hipMemcpyHostToDevice, s));
    const int64_t nt = std::max(oov, o);
    hipLaunchKernelGGL(diag_kernel, dim3(unsigned((nt + 255) / 256)), dim3(256), 0, s, c->diag.as<double>(), o,
                       v, op, kp, c->Foo.as<double>(), c->Fvv.as<double>(), c->Woooo.as<double>(),
                       c->Wvo.as<double>(), c->Wov.as<double>(), ovov.p, t2);
    GFCC_HIP(hipGetLastError());
    GFCC_HIP(hipStreamSynchronize(s));  // `ones` is pageable host memory
  }

  // ---- left vectors c_q (rows of [o][Dp])
  //  c(1h)[q,i]      = d_qi - sum_a l_ia t_qa - sum_jab (2 l_ij^ab - l_ij^ba) t_qj^ab
  //  c(2h1p)[q,k,l,c] = 2 d_qk l_lc - d_ql l_kc - sum_a t_qa (2 l_kl^ac - l_kl^ca)
  c->left.ensure(o * Dp * 8, s);
  {
    double* Cq = c->left.as<double>();
    TView L1 = tview(l1, {o, v});
    TView L2 = tview(l2, {o, o, v, v});
    DBuf b_ul;
    b_ul.ensure(n_oovv * 8, s);
    TView ul = tview(b_ul.as<double>(), {o, o, v, v});
    const int id[4] = {0, 1, 2, 3}, sw[4] = {0, 1, 3, 2};
    permute(L2, id, 2.0, ul, 0.0, s);
    permute(L2, sw, -1.0, ul, 1.0, s);
    add_diag(Cq, o, Dp + 1, nullptr, 1.0, 0.0, s);
    TView c1 = tview_s(Cq, {o, o}, {Dp, 1});  // [q][i]
    ein("ia,qa->qi", -1.0, L1, T1, 1.0, c1, scr, s);
    ein("ijab,qjab->qi", -1.0, ul, T2, 1.0, c1, scr, s);
    TView lb = tview_s(l1, {o, o, v}, {0, v, 1});
    const int id3[3] = {0, 1, 2};
    TView dk = tview_s(Cq + op, {o, o, v}, {Dp + ov, v, 1});  // q = k: [q][l][c]
    permute(lb, id3, 2.0, dk, 1.0, s);
    TView dl = tview_s(Cq + op, {o, o, v}, {Dp + v, ov, 1});  // q = l: [q][k][c]
    permute(lb, id3, -1.0, dl, 1.0, s);
    TView c2 = tview_s(Cq + op, {o, o, o, v}, {Dp, ov, v, 1});  // [q][k][l][c]
    ein("qa,klac->qklc", -1.0, T1, ul, 1.0, c2, scr, s);
    GFCC_HIP(hipStreamSynchronize(s));  // temporaries are freed on return
  }
  // ---- amplitudes for virtual-orbital right-hand sides and left vectors
  c->t1c.ensure(ov * 8, s);
  c->l1c.ensure(ov * 8, s);
  GFCC_HIP(hipMemcpyAsync(c->t1c.p, t1, size_t(ov) * 8, hipMemcpyDeviceToDevice, s));
  GFCC_HIP(hipMemcpyAsync(c->l1c.p, l1, size_t(ov) * 8, hipMemcpyDeviceToDevice, s));
  if (l2 != t2) {  // keep l2 only when it differs from t2 (Lambda = T^dagger reuses TW)
    DBuf dflag;
    dflag.ensure(sizeof(int), s);
    GFCC_HIP(hipMemsetAsync(dflag.p, 0, sizeof(int), s));
    hipLaunchKernelGGL(differ_kernel, dim3(1024), dim3(256), 0, s, l2, t2, n_oovv, dflag.as<int>());
    GFCC_HIP(hipGetLastError());
    int differ = 0;
    GFCC_HIP(hipMemcpyAsync(&differ, dflag.p, sizeof(int), hipMemcpyDeviceToHost, s));
    GFCC_HIP(hipStreamSynchronize(s));
    if (differ) {
      c->l2c.ensure(n_oovv * 8, s);
      GFCC_HIP(hipMemcpyAsync(c->l2c.p, l2, size_t(n_oovv) * 8, hipMemcpyDeviceToDevice, s));
    }
  }
  GFCC_HIP(hipStreamSynchronize(s));
  // the contraction engine's staging buffers hold integral-sized copies; the solver needs
  // only small split-K partials from them, so give the memory back
  for (auto& b : scr.b) b.release();
  (void)ovv;
}

// Reduced-precision copies of the two-body operands with power-of-two scales.
void build_lowprec(gfcc_ctx* c, int which, hipStream_t s) {
  auto& L = c->lp[which];
  if (L.built) return;
  const Prec p = which == 0 ? Prec::F32 : Prec::BF16;
  const int64_t esz = which == 0 ? 4 : 2;
  auto mk = [&](DBuf& dst, const DBuf& src, int64_t n, double& scale) {
    const double am = amax_host(src.as<double>(), n, s, c->scr);
    scale = (am > 0.0) ? std::ldexp(1.0, -std::ilogb(am)) : 1.0;  // amax -> [1, 2)
    dst.ensure(size_t(n * esz), s);
    convert_f64(src.as<double>(), dst.p, p, n, scale, s);
  };
  const int64_t ov = c->ov;
  mk(L.X1, c->X1, ov * c->kp, L.sX1);
  mk(L.Wvo, c->Wvo, ov * c->kp, L.sWvo);
  mk(L.Wov, c->Wov, ov * c->kp, L.sWov);
  mk(L.W4T, c->W4T, c->oo * c->op2, L.sW4T);
  mk(L.Zm, c->Zm, c->v * c->ldz, L.sZm);
  mk(L.TW, c->TW, c->oov * c->ktw, L.sTW);
  GFCC_HIP(hipStreamSynchronize(s));
  L.built = true;
}

}  // namespace gfcc

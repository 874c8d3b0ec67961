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
//
// Memory.  Nothing of size o^2 v^2 is held besides the ring matrix itself: every term
// whose integral factorises as (me|..)(..) in the ring's (j,a) x (m,e) pairing is a
// K = Q product through the Cholesky vectors (the t1 terms collapse into the
// factors: with P[Q,m,j] = sum_f L[Q,m,f] t_jf, Y[Q,a,j] = sum_f L[Q,a,f] t_jf and
// Tt[Q,a,e] = sum_n t_na L[Q,n,e],
//   Wovvo[m,a,e,j] <- sum_Q L[Q,m,e] (L[Q,j,a] + Z[j,a,Q] + Y[Q,a,j] - sum_n t_na (L + P)[Q,n,j]),
//   Wovov[m,a,j,e] <- sum_Q (L + P)[Q,m,j] (L - Tt)[Q,a,e],
//   Z[j,a,Q] = sum_nf (2 t_jn^af - t_jn^fa) L[Q,n,f]),
// and the exchange terms with (mf|ne) run in chunks of m (integral block) and j
// (amplitude block).  Chunk sizes follow the free device memory.  T2 (and a given
// Lambda2) are the caller's buffers; they are read in place and never copied whole.
// The pair symmetry t_ij^ab = t_ji^ba (and l_ij^ab = l_ji^ba) of closed-shell
// amplitudes is used to read t2/l2 rows in the order a product needs.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "ctx.h"

namespace gfcc {

// ------------------------------------------------------------------ memory plan

MemPlan plan_memory(int64_t o, int64_t v, int64_t Q, int prec, int restart, int flexible, int64_t window,
                    bool lambda_given) {
  MemPlan p{};
  const double d = 8.0;
  const double ov = double(o) * v, oo = double(o) * o, oov = oo * v;
  const double kp = double(round_up(int64_t(ov), 8)), Qp = double(round_up(Q, 8));
  const double op = double(round_up(o, 8)), op2 = double(round_up(int64_t(oo), 8));
  const double Dp = op + double(round_up(int64_t(oov), 8));
  const double n = double(o + v);
  p.input_L = Q * n * n * d;
  p.input_t2 = oov * v * d;
  p.input_l2 = lambda_given ? p.input_t2 : 0.0;
  p.ring = ov * 2.0 * kp * d;
  p.ladder = oo * op2 * d;
  p.wovoo = oov * op * d;
  p.wooov = oov * o * d;
  p.chol = (Q * kp + v * o * Qp) * d;
  p.rows_1h = o * Dp * d;
  p.left = o * Dp * d;
  p.vectors = (2.0 * Dp + oov) * d;  // diagonal, d1b and the rest of O(D)
  p.small = (oo + v * v + 3.0 * ov) * d;
  p.context_fp64 = p.ring + p.ladder + p.wovoo + p.wooov + p.chol + p.rows_1h + p.left + p.vectors + p.small;
  const double esz = (prec == GFCC_BF16_IR || prec == GFCC_FP16_IR) ? 2.0 : (prec == GFCC_FP32_IR ? 4.0 : 0.0);
  p.context_lowp = esz * (ov * 2.0 * kp + oo * op2 + oov * op + oov * v + Q * kp);
  // build temporaries: seven Q-innermost (o v) x Q or o^2 x Q factors and two o^3 v blocks;
  // chunk buffers come on top and shrink to fit
  p.build_fixed = (5.0 * ov * Qp + 4.0 * oo * Qp) * d + 2.0 * oov * o * d;
  p.build_chunk_min = 3.0 * v * ov * d;  // one occupied index of the largest chunked phase
  const int m = std::min(std::max(restart, 1), 64);
  // Krylov basis (and flexible-GMRES Z), solution, one spare plane pair, sigma input/output planes
  p.per_slot = (double(m + 2 + (flexible ? m : 0)) * 2.0 + 4.0) * Dp * d;
  // sigma operand copies for the 2 planes of each window slot, sized for the FP64 sigma of the
  // true residual (the largest): [2R - RT | -R], RT, the ladder operand, U and z
  const double P = 2.0 * double(window);
  p.sigma_ws = P * d * (o * 3.0 * kp + v * op2 + o * Qp + 2.0 * double(round_up(v, 8)) + op);
  p.total = p.input_t2 + p.input_l2 + p.context_fp64 + p.context_lowp + double(window) * p.per_slot + p.sigma_ws;
  p.build_peak = p.input_L + p.input_t2 + p.input_l2 + p.context_fp64 + p.build_fixed + p.build_chunk_min;
  return p;
}

namespace {

// FP64 product C(i,j) = alpha sum_k A(i,k) B(j,k) + beta C(i,j) (see GemmArgs); large
// products on the 128x256 tile with direct-to-LDS loads, small grids split along K.
void g64(const GemmArgs& g, Scratch& scr, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return;
  if (g.batch == 1 && !g.b_ncontig && g.M >= 1024 && g.N >= 1024)
    gemm(Prec::F64, g, TILE_DMA2_128x256, s);
  else if (g.batch == 1)
    gemm_auto(Prec::F64, g, scr, 3, s);
  else
    gemm(Prec::F64, g, gemm_default_cfg(g.M, g.N, g.K), s);
}

GemmArgs mk(const double* A, RowMap am, const double* B, RowMap bm, double* C, RowMap cm, RowMap cn, int64_t M,
            int64_t N, int64_t K, double alpha, double beta) {
  GemmArgs g;
  g.A = A;
  g.am = am;
  g.B = B;
  g.bm = bm;
  g.C = C;
  g.cm = cm;
  g.cn = cn;
  g.M = M;
  g.N = N;
  g.K = K;
  g.alpha = alpha;
  g.beta = beta;
  return g;
}

__global__ void add_diag_kernel(double* p, int64_t n, int64_t stride, const double* src, double alpha,
                                double beta) {
  int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < n) p[t * stride] = beta * p[t * stride] + alpha * (src ? src[t] : 1.0);
}

void add_diag(double* p, int64_t n, int64_t stride, const double* src, double alpha, double beta, hipStream_t s) {
  hipLaunchKernelGGL(add_diag_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, p, n, stride, src, alpha,
                     beta);
  GFCC_HIP(hipGetLastError());
}

// y = a x + b y over n elements
__global__ void axpby_kernel(double* __restrict__ y, const double* __restrict__ x, int64_t n, double a, double b) {
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n; t += int64_t(gridDim.x) * blockDim.x)
    y[t] = a * x[t] + b * y[t];
}

void axpby(double* y, const double* x, int64_t n, double a, double b, hipStream_t s) {
  if (n <= 0) return;
  const unsigned nb = unsigned(std::min<int64_t>((n + 255) / 256, 65536));
  hipLaunchKernelGGL(axpby_kernel, dim3(nb), dim3(256), 0, s, y, x, n, a, b);
  GFCC_HIP(hipGetLastError());
}

// flag = 1 when a[0:n] and b[0:n] differ anywhere
__global__ void differ_kernel(const double* __restrict__ a, const double* __restrict__ b, int64_t n, int* flag) {
  bool dif = false;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n; t += int64_t(gridDim.x) * blockDim.x)
    dif = dif || (a[t] != b[t]);
  if (dif) *flag = 1;
}

// Exact diagonal of the 2h1p block for i in [i0, i0 + ci), with the integral chunk
// B[(i - i0, j)][(e, f)] = (ie|jf).  WW rows (j,a): Wovvo at column (m,e), Wovov at kp + (m,e).
__global__ void diag_kernel(double* __restrict__ dg, int64_t o, int64_t v, int64_t o_pad, int64_t kp, int64_t k2,
                            int64_t op2, int64_t i0, int64_t ci, const double* __restrict__ Foo,
                            const double* __restrict__ Fvv, const double* __restrict__ W4T,
                            const double* __restrict__ WW, const double* __restrict__ Bc,
                            const double* __restrict__ t2) {
  const int64_t ov = o * v, vv = v * v;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;  // (i - i0, j, a)
  if (t >= ci * ov) return;
  const int64_t a = t % v, j = (t / v) % o, i = i0 + t / ov;
  auto wvo = [&](int64_t m, int64_t aa, int64_t e, int64_t jj) { return WW[(jj * v + aa) * k2 + m * v + e]; };
  auto wov = [&](int64_t m, int64_t aa, int64_t jj, int64_t e) { return WW[(jj * v + aa) * k2 + kp + m * v + e]; };
  double dv = Fvv[a * v + a] - Foo[i * o + i] - Foo[j * o + j];
  dv += W4T[(i * o + j) * op2 + i * o + j];
  dv += 2.0 * wvo(j, a, a, j) - wov(j, a, j, a);
  if (i == j) dv -= wvo(i, a, a, i);
  dv -= wov(i, a, i, a);
  const double* brow = Bc + ((i - i0) * o + j) * vv;
  const double* trow = t2 + (i * o + j) * vv;
  double tb = 0.0;
  for (int64_t e = 0; e < v; ++e) {
    const double g1 = brow[e * v + a];  // (ie|ja)
    const double g2 = brow[a * v + e];  // (ia|je)
    tb += (2.0 * g1 - g2) * trow[e * v + a];
  }
  dg[o_pad + i * ov + j * v + a] = dv - tb;
}

// (1h) diagonal: -Foo[i,i]
__global__ void diag1_kernel(double* __restrict__ dg, const double* __restrict__ Foo, int64_t o) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < o) dg[t] = -Foo[t * o + t];
}

int64_t clamp_chunk(double avail, double per_unit, int64_t hi) {
  const double c = per_unit > 0.0 ? std::floor(avail / per_unit) : double(hi);
  return std::max<int64_t>(1, std::min<int64_t>(hi, int64_t(c)));
}

}  // namespace

void build_intermediates(gfcc_ctx* c, const gfcc_system* sys, hipStream_t s) {
  const int64_t o = c->o, v = c->v, Q = c->Q, n = c->n;
  const int64_t ov = c->ov, oo = c->oo, oov = c->oov, vv = v * v;
  const int64_t kp = c->kp, k2 = c->k2, op = c->o_pad, op2 = c->op2, Qp = c->Qp, Dp = c->Dp;
  const int64_t nn = n * n;
  Scratch& scr = c->scr;
  const double* L = sys->L;
  const double* t1 = sys->t1;
  const double* t2 = sys->t2;
  const double* l1 = sys->l1 ? sys->l1 : sys->t1;
  const double* eps = sys->eps;
  c->t2 = t2;
  c->l2 = nullptr;
  const bool verbose = std::getenv("GFCC_VERBOSE") != nullptr;

  // ---- persistent blocks (zero-filled)
  {
    const MemPlan plan = plan_memory(o, v, Q, GFCC_FP64, 30, 0, 0, sys->l2 != nullptr);
    if (verbose)
      std::fprintf(stderr,
                   "[gfcc] o=%lld v=%lld Q=%lld: ring %.2f GB, ladder %.2f, Wovoo %.2f, Wooov %.2f, Cholesky %.2f, "
                   "1h rows %.2f, left %.2f, vectors %.2f -> context %.2f GB (FP64); build temporaries %.2f GB + "
                   "chunks; caller's t2 %.2f GB stays borrowed\n",
                   (long long)o, (long long)v, (long long)Q, plan.ring / 1e9, plan.ladder / 1e9, plan.wovoo / 1e9,
                   plan.wooov / 1e9, plan.chol / 1e9, plan.rows_1h / 1e9, plan.left / 1e9, plan.vectors / 1e9,
                   plan.context_fp64 / 1e9, plan.build_fixed / 1e9, plan.input_t2 / 1e9);
  }
  c->WW.ensure(size_t(ov * k2) * 8, s);
  c->W4T.ensure(size_t(oo * op2) * 8, s);
  c->WovooT.ensure(size_t(oov * op) * 8, s);
  c->Wooov.ensure(size_t(oov * o) * 8, s);
  c->LovC.ensure(size_t(Q * kp) * 8, s);
  c->LovT.ensure(size_t(v * o * Qp) * 8, s);
  c->Foo.ensure(size_t(oo) * 8, s);
  c->Fvv.ensure(size_t(vv) * 8, s);
  c->Fov.ensure(size_t(ov) * 8, s);
  c->d1b.ensure(size_t(oov) * 8, s);
  c->Uop.ensure(size_t(o * Dp) * 8, s);
  c->diag.ensure(size_t(Dp) * 8, s);
  c->left.ensure(size_t(o * Dp) * 8, s);
  c->t1c.ensure(size_t(ov) * 8, s);
  c->l1c.ensure(size_t(ov) * 8, s);
  double* WW = c->WW.as<double>();
  double* W4T = c->W4T.as<double>();
  double* WovooT = c->WovooT.as<double>();
  double* Wooov = c->Wooov.as<double>();
  double* LovC = c->LovC.as<double>();
  double* LovT = c->LovT.as<double>();
  double* Foo = c->Foo.as<double>();
  double* Fvv = c->Fvv.as<double>();
  double* Fov = c->Fov.as<double>();

  // ---- temporaries of the build
  DBuf b_LovQ, b_LooQ, b_LP, b_PQ, b_YQ, b_Z, b_ZT, b_LooT, b_AV, b_xQ, b_t1T, b_ooov, b_S;
  b_LovQ.ensure(size_t(ov * Qp) * 8, s);  // [(m,e)][Q] = L[Q][m][o+e]
  b_LooQ.ensure(size_t(oo * Qp) * 8, s);  // [(m,i)][Q] = L[Q][m][i]
  b_LP.ensure(size_t(oo * Qp) * 8, s);    // [(m,i)][Q] = L[Q][m][i] + P[Q][m][i]
  b_PQ.ensure(size_t(oo * Qp) * 8, s);    // [(m,j)][Q] = P[Q][m][j] = sum_f L[Q][m][o+f] t_jf
  b_YQ.ensure(size_t(ov * Qp) * 8, s);    // [(a,j)][Q] = Y[Q][a][j] = sum_f L[Q][o+a][o+f] t_jf
  b_Z.ensure(size_t(ov * Qp) * 8, s);     // [(i,e)][Q] = Z[i,e,Q]
  b_ZT.ensure(size_t(ov * Qp) * 8, s);    // [e][(i,Q)]
  b_LooT.ensure(size_t(oo * Qp) * 8, s);  // [i][(n,Q)] = L[Q][n][i]
  b_AV.ensure(size_t(ov * Qp) * 8, s);    // [(j,a)][Q] Coulomb factor of the Wovvo ring block
  b_xQ.ensure(size_t(Qp) * 8, s);
  b_t1T.ensure(size_t(v * op) * 8, s);    // [a][n] = t1[n][a] (row stride o_pad)
  b_ooov.ensure(size_t(oov * o) * 8, s);  // [(m,i)][(n,e)] = (mi|ne)
  double* LovQ = b_LovQ.as<double>();
  double* LooQ = b_LooQ.as<double>();
  double* LP = b_LP.as<double>();
  double* PQ = b_PQ.as<double>();
  double* YQ = b_YQ.as<double>();
  double* Z = b_Z.as<double>();
  double* ZT = b_ZT.as<double>();
  double* LooT = b_LooT.as<double>();
  double* AV = b_AV.as<double>();
  double* xQ = b_xQ.as<double>();
  double* t1T = b_t1T.as<double>();
  double* ooov = b_ooov.as<double>();

  // chunk budget: what is left of free memory after the fixed temporaries
  size_t freeb = 0, totalb = 0;
  GFCC_HIP(hipMemGetInfo(&freeb, &totalb));
  const double avail = std::max(0.0, 0.85 * double(freeb) - double(oov * o) * 8.0 - 2.0e9);
  if (verbose) std::fprintf(stderr, "[gfcc] free %.2f GB, chunk budget %.2f GB\n", freeb / 1e9, avail / 1e9);

  const int id2[2] = {0, 1}, id3[3] = {0, 1, 2}, id4[4] = {0, 1, 2, 3};
  TView T1 = tview(const_cast<double*>(t1), {o, v});

  // ================================================================= Cholesky factors
  permute(tview_s(const_cast<double*>(L) + o, {Q, o, v}, {nn, n, 1}), id3, 1.0, tview_s(LovQ, {Q, o, v}, {1, v * Qp, Qp}),
          0.0, s);
  permute(tview_s(const_cast<double*>(L), {Q, o, o}, {nn, n, 1}), id3, 1.0, tview_s(LooQ, {Q, o, o}, {1, o * Qp, Qp}),
          0.0, s);
  permute(tview_s(const_cast<double*>(L) + o, {Q, o, v}, {nn, n, 1}), id3, 1.0, tview_s(LovC, {Q, o, v}, {kp, v, 1}),
          0.0, s);
  permute(tview_s(const_cast<double*>(L) + o, {Q, o, v}, {nn, n, 1}), id3, 1.0, tview_s(LovT, {Q, o, v}, {1, Qp, o * Qp}),
          0.0, s);
  permute(tview_s(const_cast<double*>(L), {Q, o, o}, {nn, n, 1}), id3, 1.0, tview_s(LooT, {Q, o, o}, {1, Qp, o * Qp}),
          0.0, s);
  permute(T1, std::array<int, 2>{1, 0}.data(), 1.0, tview_s(t1T, {v, o}, {op, 1}), 0.0, s);
  // xQ[Q] = sum_mf t_mf L[Q][m][o+f]
  g64(mk(t1, lin(0), LovC, lin(kp), xQ, lin(0), lin(1), 1, Q, ov, 1.0, 0.0), scr, s);
  // PQ[(m,j)][Q] = sum_f t1[j][f] L[Q][m][o+f]: per m, B = LovQ rows (m,f) as K-rows (N = Q contiguous)
  {
    GemmArgs g = mk(t1, lin(v), LovQ, lin(Qp), PQ, lin(Qp), lin(1), o, Q, v, 1.0, 0.0);
    g.b_ncontig = 1;
    g.batch = int(o);
    g.bz = lin(v * Qp);
    g.cz = lin(o * Qp);
    g64(g, scr, s);
  }
  // LP = LooQ + PQ
  GFCC_HIP(hipMemcpyAsync(LP, LooQ, size_t(oo * Qp) * 8, hipMemcpyDeviceToDevice, s));
  axpby(LP, PQ, oo * Qp, 1.0, 1.0, s);

  // ================================================================= Z[i,e,Q] = sum_nf u2[i,n,e,f] L[Q][n][o+f]
  {
    const int64_t ci = clamp_chunk(avail, double(v * ov) * 8.0, o);
    DBuf b_u;
    b_u.ensure(size_t(ci * v * kp) * 8, s);
    double* U = b_u.as<double>();
    for (int64_t i0 = 0; i0 < o; i0 += ci) {
      const int64_t cn_ = std::min(ci, o - i0);
      // U[(i,e)][(n,f)] = 2 t2[i,n,e,f] - t2[i,n,f,e]
      TView src = tview_s(const_cast<double*>(t2) + i0 * o * vv, {cn_, v, o, v}, {o * vv, v, vv, 1});   // i e n f
      TView srs = tview_s(const_cast<double*>(t2) + i0 * o * vv, {cn_, v, o, v}, {o * vv, 1, vv, v});   // t2[i,n,f,e]
      TView dst = tview_s(U, {cn_, v, o, v}, {v * kp, kp, v, 1});
      permute(src, id4, 2.0, dst, 0.0, s);
      permute(srs, id4, -1.0, dst, 1.0, s);
      g64(mk(U, lin(kp), LovC, lin(kp), Z + i0 * v * Qp, lin(Qp), lin(1), cn_ * v, Q, ov, 1.0, 0.0), scr, s);
    }
    GFCC_HIP(hipStreamSynchronize(s));
  }
  permute(tview_s(Z, {o, v, Q}, {v * Qp, Qp, 1}), id3, 1.0, tview_s(ZT, {o, v, Q}, {Qp, o * Qp, 1}), 0.0, s);

  // ================================================================= one-body blocks (part 1)
  // Fov[m,e] = 2 sum_Q L[Q,m,e] xQ[Q] - sum_(n,Q) P[Q,m,n] L[Q,n,e]
  g64(mk(LovQ, lin(Qp), xQ, lin(0), Fov, lin(1), lin(0), ov, 1, Q, 2.0, 0.0), scr, s);
  g64(mk(PQ, lin(o * Qp), LovT, lin(o * Qp), Fov, lin(v), lin(1), o, v, o * Qp, -1.0, 1.0), scr, s);
  // Foo[m,i] = e_i d_mi + sum_e t_ie Fov[m,e] + 2 sum_Q L[Q,m,i] xQ[Q] - sum_(n,Q) P[Q,m,n] L[Q,n,i]
  //            + sum_(e,Q) L[Q,m,e] Z[i,e,Q]
  add_diag(Foo, o, o + 1, eps, 1.0, 0.0, s);
  g64(mk(Fov, lin(v), t1, lin(v), Foo, lin(o), lin(1), o, o, v, 1.0, 1.0), scr, s);
  g64(mk(LooQ, lin(Qp), xQ, lin(0), Foo, lin(1), lin(0), oo, 1, Q, 2.0, 1.0), scr, s);
  g64(mk(PQ, lin(o * Qp), LooT, lin(o * Qp), Foo, lin(o), lin(1), o, o, o * Qp, -1.0, 1.0), scr, s);
  g64(mk(LovQ, lin(v * Qp), Z, lin(v * Qp), Foo, lin(o), lin(1), o, o, v * Qp, 1.0, 1.0), scr, s);
  // Fvv[a,e] = e_a d_ae - sum_m t_ma Fov[m,e] - sum_(m,Q) Z[m,a,Q] L[Q,m,e]
  //            (+ 2 sum_Q xQ L[Q,a,e] - sum_(m,Q) Y[Q,a,m] L[Q,m,e] in the virtual-chunk loop)
  add_diag(Fvv, v, v + 1, eps + o, 1.0, 0.0, s);
  {
    // - sum_m t1[m][a] Fov[m][e] (small blocks)
    TView FovV = tview(Fov, {o, v});
    TView FvvV = tview(Fvv, {v, v});
    ein("ma,me->ae", -1.0, T1, FovV, 1.0, FvvV, scr, s);
  }
  g64(mk(ZT, lin(o * Qp), LovT, lin(o * Qp), Fvv, lin(v), lin(1), v, v, o * Qp, -1.0, 1.0), scr, s);

  // ================================================================= virtual-chunk loop
  // per chunk of a: LvvQ_c[(a,f)][Q] = L[Q][o+a][o+f]
  //   Y[Q,a,j]                      -> YQ
  //   Fvv += 2 sum_Q L[Q,a,e] xQ
  //   Wovoo[m,a,i,j] += sum_ef (me|af) t2[i,j,e,f]   (G_c[(m,a)][(e,f)] = (me|af))
  //   Wovov[m,a,j,e] = sum_Q (L + P)[Q,m,j] (L - Tt)[Q,a,e]
  {
    const double per_a = double(v * Qp) * 8.0 + double(o * vv) * 8.0;
    const int64_t ca = clamp_chunk(avail, per_a, v);
    DBuf b_lvv, b_g;
    b_lvv.ensure(size_t(ca * v * Qp) * 8, s);
    b_g.ensure(size_t(o * ca * vv) * 8, s);
    double* Lvc = b_lvv.as<double>();
    double* Gc = b_g.as<double>();
    for (int64_t a0 = 0; a0 < v; a0 += ca) {
      const int64_t na = std::min(ca, v - a0);
      permute(tview_s(const_cast<double*>(L) + (o + a0) * n + o, {Q, na, v}, {nn, n, 1}), id3, 1.0,
              tview_s(Lvc, {Q, na, v}, {1, v * Qp, Qp}), 0.0, s);
      // YQ[(a,j)][Q] = sum_f t1[j][f] Lvc[(a,f)][Q]  (batched over a, B N-contiguous)
      {
        GemmArgs g = mk(t1, lin(v), Lvc, lin(Qp), YQ + a0 * o * Qp, lin(Qp), lin(1), o, Q, v, 1.0, 0.0);
        g.b_ncontig = 1;
        g.batch = int(na);
        g.bz = lin(v * Qp);
        g.cz = lin(o * Qp);
        g64(g, scr, s);
      }
      // Fvv[a][e] += 2 sum_Q Lvc[(a,e)][Q] xQ[Q]
      g64(mk(Lvc, lin(Qp), xQ, lin(0), Fvv + a0 * v, lin(1), lin(0), na * v, 1, Q, 2.0, 1.0), scr, s);
      // G_c[(m,a)][(e,f)] = sum_Q LovQ[(m,e)][Q] Lvc[(a,f)][Q]
      g64(mk(LovQ, lin(Qp), Lvc, lin(Qp), Gc, two(v, na * vv, v), two(v, vv, 1), ov, na * v, Q, 1.0, 0.0), scr, s);
      // WovooT[(i,j,a)][m] += sum_(e,f) G_c[(m,a)][(e,f)] t2[(i,j)][(e,f)]
      g64(mk(Gc, lin(vv), t2, lin(vv), WovooT + a0 * op, two(na, 1, op), lin(v * op), o * na, oo, vv, 1.0, 1.0), scr,
          s);
      // Lvc -= Tt: Tt[(a,e)][Q] = sum_n t1[n][a] LovQ[(n,e)][Q]  (batched over e, B N-contiguous)
      {
        GemmArgs g = mk(t1T + a0 * op, lin(op), LovQ, lin(v * Qp), Lvc, lin(v * Qp), lin(1), na, Q, o, -1.0, 1.0);
        g.b_ncontig = 1;
        g.batch = int(v);
        g.bz = lin(Qp);
        g.cz = lin(Qp);
        g64(g, scr, s);
      }
      // Wovov block: C[(m,j)][(a,e)] = sum_Q LP[(m,j)][Q] (L - Tt)[(a,e)][Q] -> WW[(j,a)][kp + (m,e)]
      g64(mk(LP, lin(Qp), Lvc, lin(Qp), WW + kp + a0 * k2, two(o, v, v * k2), two(v, k2, 1), oo, na * v, Q, 1.0,
             0.0),
          scr, s);
    }
    GFCC_HIP(hipStreamSynchronize(s));
  }
  // Fvv[a,e] -= sum_(m,Q) Y[Q,a,m] L[Q,m,e]
  g64(mk(YQ, lin(o * Qp), LovT, lin(o * Qp), Fvv, lin(v), lin(1), v, v, o * Qp, -1.0, 1.0), scr, s);

  // ================================================================= Wovoo K = Q part and the Wovvo factor
  // AV[(j,a)][Q] = L[Q][j][o+a] + Y[Q,a,j]
  GFCC_HIP(hipMemcpyAsync(AV, LovQ, size_t(ov * Qp) * 8, hipMemcpyDeviceToDevice, s));
  permute(tview_s(YQ, {v, o, Q}, {o * Qp, Qp, 1}), id3, 1.0, tview_s(AV, {v, o, Q}, {Qp, v * Qp, 1}), 1.0, s);
  // WovooT[(i,j,a)][m] += sum_Q LP[(m,i)][Q] AV[(j,a)][Q] + sum_Q PQ[(m,i)][Q] Z[(j,a)][Q]
  g64(mk(LP, lin(Qp), AV, lin(Qp), WovooT, two(o, 1, o * v * op), lin(op), oo, ov, Q, 1.0, 1.0), scr, s);
  g64(mk(PQ, lin(Qp), Z, lin(Qp), WovooT, two(o, 1, o * v * op), lin(op), oo, ov, Q, 1.0, 1.0), scr, s);
  // AV += Z - sum_n t1[n][a] LP[(n,j)][Q]  (batched over j, B N-contiguous)
  axpby(AV, Z, ov * Qp, 1.0, 1.0, s);
  {
    GemmArgs g = mk(t1T, lin(op), LP, lin(o * Qp), AV, lin(Qp), lin(1), v, Q, o, -1.0, 1.0);
    g.b_ncontig = 1;
    g.batch = int(o);
    g.bz = lin(Qp);
    g.cz = lin(v * Qp);
    g64(g, scr, s);
  }
  // Wovvo block (Coulomb part): WW[(j,a)][(m,e)] = sum_Q AV[(j,a)][Q] L[Q][m][o+e]
  g64(mk(AV, lin(Qp), LovQ, lin(Qp), WW, lin(k2), lin(1), ov, ov, Q, 1.0, 0.0), scr, s);

  // ================================================================= exchange parts of the ring blocks
  //   WW[(j,a)][w kp + (m,e)] -= sum_(n,f) T_w[(j,a)][(n,f)] (mf|ne),
  //   T_0[(j,a)][(n,f)] = t2[j,n,a,f] (Wovvo), T_1 = t2[j,n,f,a] (Wovov)
  {
    const double per = double(v * kp) * 8.0 * 3.0;  // X_c rows of one m plus T_c rows (two blocks) of one j
    const int64_t c1 = clamp_chunk(avail, per, o);
    DBuf b_x, b_t;
    b_x.ensure(size_t(c1 * v * kp) * 8, s);
    b_t.ensure(size_t(2 * c1 * v * kp) * 8, s);
    double* Xc = b_x.as<double>();
    double* Tc = b_t.as<double>();
    for (int64_t m0 = 0; m0 < o; m0 += c1) {
      const int64_t nm = std::min(c1, o - m0);
      // X_c[(m,e)][(n,f)] = (mf|ne) = sum_Q LovQ[(m,f)][Q] LovQ[(n,e)][Q]
      g64(mk(LovQ + m0 * v * Qp, lin(Qp), LovQ, lin(Qp), Xc, two(v, v * kp, 1), two(v, v, kp), nm * v, ov, Q, 1.0,
             0.0),
          scr, s);
      for (int64_t j0 = 0; j0 < o; j0 += c1) {
        const int64_t nj = std::min(c1, o - j0);
        const double* tj = t2 + j0 * o * vv;
        // T_c[w][(j,a)][(n,f)]
        permute(tview_s(const_cast<double*>(tj), {nj, v, o, v}, {o * vv, v, vv, 1}), id4, 1.0,
                tview_s(Tc, {nj, v, o, v}, {v * kp, kp, v, 1}), 0.0, s);
        permute(tview_s(const_cast<double*>(tj), {nj, v, o, v}, {o * vv, 1, vv, v}), id4, 1.0,
                tview_s(Tc + nj * v * kp, {nj, v, o, v}, {v * kp, kp, v, 1}), 0.0, s);
        g64(mk(Tc, lin(kp), Xc, lin(kp), WW + j0 * v * k2 + m0 * v, two(nj * v, kp, k2), lin(1), 2 * nj * v, nm * v,
               ov, -1.0, 1.0),
            scr, s);
      }
    }
    GFCC_HIP(hipStreamSynchronize(s));
  }

  // ================================================================= Woooo, Wooov, ooov
  // W4T[(i,j)][(m,n)] = sum_Q LP[(m,i)][Q] LP[(n,j)][Q]   (+ the t2 term in the m-chunk loop below)
  g64(mk(LP, lin(Qp), LP, lin(Qp), W4T, two(o, o, o * op2), two(o, 1, op2), oo, oo, Q, 1.0, 0.0), scr, s);
  // Wooov[m,n,i,e] = sum_Q LP[(m,i)][Q] L[Q][n][o+e]
  g64(mk(LP, lin(Qp), LovQ, lin(Qp), Wooov, two(o, o * ov, v), two(v, ov, 1), oo, ov, Q, 1.0, 0.0), scr, s);
  // ooov[(m,i)][(n,e)] = (mi|ne)
  g64(mk(LooQ, lin(Qp), LovQ, lin(Qp), ooov, lin(ov), lin(1), oo, ov, Q, 1.0, 0.0), scr, s);

  // ================================================================= (me|nf) chunks over m:
  //   W4T[(i,j)][(m,n)] += sum_ef t2[i,j,e,f] (me|nf)  and the exact diagonal of the rows i = m
  {
    const int64_t cm = clamp_chunk(avail, double(o * vv) * 8.0, o);
    DBuf b_b;
    b_b.ensure(size_t(cm * o * vv) * 8, s);
    double* Bc = b_b.as<double>();
    for (int64_t m0 = 0; m0 < o; m0 += cm) {
      const int64_t nm = std::min(cm, o - m0);
      // Bc[(m,n)][(e,f)] = sum_Q LovQ[(m,e)][Q] LovQ[(n,f)][Q]
      g64(mk(LovQ + m0 * v * Qp, lin(Qp), LovQ, lin(Qp), Bc, two(v, o * vv, v), two(v, vv, 1), nm * v, ov, Q, 1.0,
             0.0),
          scr, s);
      g64(mk(t2, lin(vv), Bc, lin(vv), W4T + m0 * o, lin(op2), lin(1), oo, nm * o, vv, 1.0, 1.0), scr, s);
    }
    GFCC_HIP(hipStreamSynchronize(s));
  }

  // ================================================================= Wovoo: remaining terms
  // Fov term: WovooT[(i,j,a)][m] += sum_e t2[j,i,a,e] Fov[m,e]   (t_ij^ea = t_ji^ae; batched over j)
  {
    GemmArgs g = mk(t2, two(v, vv, v), Fov, lin(v), WovooT, two(v, o * v * op, op), lin(1), ov, o, v, 1.0, 1.0);
    g.batch = int(o);
    g.az = lin(o * vv);
    g.cz = lin(v * op);
    g64(g, scr, s);
  }
  // - sum_n t1[n][a] Woooo[m,n,i,j]: C[a][(i,j,m)] with B rows (i,j,m) of W4T (K = n)
  g64(mk(t1T, lin(op), W4T, two(o, op2, o), WovooT, lin(op), two(o, v * op, 1), v, oo * o, o, -1.0, 1.0), scr, s);
  // o^3 v^2 terms:  S[(m,i)][(n,f)] = sum_Q L[Q][m][o+f] P[Q][n][i] = sum_e t_ie (mf|ne);
  //   AS[(m,i)][(n,e)] = (me|ni) + S[(m,i)][(n,e)]
  //   WovooT += ooov[(m,i)] u2[j,n,a,e] - AS[(m,i)] t2[j,n,a,e]   (rows (m,i), columns (j,a))
  //   WovooT -= AS[(m,j)] t2[i,n,e,a]                            (rows (m,j), columns (i,a))
  {
    b_S.ensure(size_t(oov * o) * 8, s);
    double* AS = b_S.as<double>();
    // S: C[(m,f)][(n,i)] = sum_Q LovQ[(m,f)][Q] PQ[(n,i)][Q] -> AS[(m,i)][(n,f)]
    g64(mk(LovQ, lin(Qp), PQ, lin(Qp), AS, two(v, o * ov, 1), two(o, v, ov), ov, oo, Q, 1.0, 0.0), scr, s);
    // + (me|ni) = ooov[n,i,m,e]
    permute(tview_s(ooov, {o, o, o, v}, {v, ov, o * ov, 1}), id4, 1.0, tview_s(AS, {o, o, o, v}, {o * ov, ov, v, 1}),
            1.0, s);
    const int64_t cj = clamp_chunk(avail, 3.0 * double(v * kp) * 8.0, o);
    DBuf b_c;
    b_c.ensure(size_t(3 * cj * v * kp) * 8, s);
    double* T2c = b_c.as<double>();
    double* T3c = T2c + cj * v * kp;
    double* U2c = T3c + cj * v * kp;
    for (int64_t j0 = 0; j0 < o; j0 += cj) {
      const int64_t nj = std::min(cj, o - j0);
      const double* tj = t2 + j0 * o * vv;
      // T2c[(j,a)][(n,e)] = t2[j,n,a,e];  T3c[(j,a)][(n,e)] = t2[j,n,e,a];  U2c = 2 T2c - T3c
      permute(tview_s(const_cast<double*>(tj), {nj, v, o, v}, {o * vv, v, vv, 1}), id4, 1.0,
              tview_s(T2c, {nj, v, o, v}, {v * kp, kp, v, 1}), 0.0, s);
      permute(tview_s(const_cast<double*>(tj), {nj, v, o, v}, {o * vv, 1, vv, v}), id4, 1.0,
              tview_s(T3c, {nj, v, o, v}, {v * kp, kp, v, 1}), 0.0, s);
      GFCC_HIP(hipMemcpyAsync(U2c, T3c, size_t(nj * v * kp) * 8, hipMemcpyDeviceToDevice, s));
      axpby(U2c, T2c, nj * v * kp, 2.0, -1.0, s);
      double* Cj = WovooT + j0 * v * op;
      g64(mk(ooov, lin(ov), U2c, lin(kp), Cj, two(o, 1, o * v * op), lin(op), oo, nj * v, ov, 1.0, 1.0), scr, s);
      g64(mk(AS, lin(ov), T2c, lin(kp), Cj, two(o, 1, o * v * op), lin(op), oo, nj * v, ov, -1.0, 1.0), scr, s);
      // rows (m,j) of AS against the chunk as the i index: WovooT[(i,j,a)][m]
      g64(mk(AS, lin(ov), T3c, lin(kp), WovooT + j0 * o * v * op, two(o, 1, v * op), two(v, o * v * op, op), oo,
             nj * v, ov, -1.0, 1.0),
          scr, s);
    }
    GFCC_HIP(hipStreamSynchronize(s));
  }
  b_S.release();
  b_ooov.release();

  // ================================================================= one-body folds, d1b, diagonal
  // Fold the off-diagonal one-body terms into the Wovov block (exact):
  //   WW[(j,a)][kp + (m,e)] += Foo_off[m,j] d_ae - 1/2 Fvv_off[a,e] d_jm
  // Sigma reads this block twice (-[Wovov] R in the first ring product, rows (i) x cols (j,a),
  // and -[Wovov] RT in the second): the Foo fold gives -sum_m Foo_off[m,j] r[i][m][a] through
  // the first and -sum_m Foo_off[m,i] r[m][j][a] through the second; the Fvv fold gives half of
  // sum_e Fvv_off[a,e] r[i][j][e] through each.  The diagonal one-body part
  // (Fvv[a,a] - Foo[i,i] - Foo[j,j]) r[i][j][a] is applied elementwise in FP64 by sigma.
  {
    double* Wv = WW + kp;
    TView foo_b = tview_s(Foo, {o, v, o}, {1, 0, o});                 // [j][a][m] -> Foo[m][j]
    TView foo_d = tview_s(Foo, {o, v}, {o + 1, 0});                   // [j][a]    -> Foo[j][j]
    TView w_ae = tview_s(Wv, {o, v, o}, {v * k2, k2 + 1, v});         // [j][a][m], e = a
    TView w_d = tview_s(Wv, {o, v}, {v * k2 + v, k2 + 1});            // [j][a],    m = j, e = a
    permute(foo_b, id3, 1.0, w_ae, 1.0, s);
    permute(foo_d, id2, -1.0, w_d, 1.0, s);
    TView fvv_b = tview_s(Fvv, {o, v, v}, {0, v, 1});                 // [j][a][e] -> Fvv[a][e]
    TView fvv_d = tview_s(Fvv, {o, v}, {0, v + 1});                   // [j][a]    -> Fvv[a][a]
    TView w_jm = tview_s(Wv, {o, v, v}, {v * k2 + v, k2, 1});         // [j][a][e], m = j
    permute(fvv_b, id3, -0.5, w_jm, 1.0, s);
    permute(fvv_d, id2, 0.5, w_d, 1.0, s);
  }
  {
    TView out = tview(c->d1b.as<double>(), {o, o, v});
    permute(tview_s(Fvv, {o, o, v}, {0, 0, v + 1}), id3, 1.0, out, 0.0, s);
    permute(tview_s(Foo, {o, o, v}, {o + 1, 0, 0}), id3, -1.0, out, 1.0, s);
    permute(tview_s(Foo, {o, o, v}, {0, o + 1, 0}), id3, -1.0, out, 1.0, s);
  }
  // exact diagonal (padding 1 so that Jacobi keeps zeros); the 2h1p part per chunk of i with (ie|jf)
  {
    std::vector<double> ones(size_t(Dp), 1.0);
    GFCC_HIP(hipMemcpyAsync(c->diag.p, ones.data(), size_t(Dp) * 8, hipMemcpyHostToDevice, s));
    GFCC_HIP(hipStreamSynchronize(s));  // `ones` is pageable host memory
    double* dg = c->diag.as<double>();
    hipLaunchKernelGGL(diag1_kernel, dim3(unsigned((o + 255) / 256)), dim3(256), 0, s, dg, Foo, o);
    GFCC_HIP(hipGetLastError());
    const int64_t ci = clamp_chunk(avail, double(o * vv) * 8.0, o);
    DBuf b_b;
    b_b.ensure(size_t(ci * o * vv) * 8, s);
    double* Bc = b_b.as<double>();
    for (int64_t i0 = 0; i0 < o; i0 += ci) {
      const int64_t ni = std::min(ci, o - i0);
      g64(mk(LovQ + i0 * v * Qp, lin(Qp), LovQ, lin(Qp), Bc, two(v, o * vv, v), two(v, vv, 1), ni * v, ov, Q, 1.0,
             0.0),
          scr, s);
      const int64_t nt = ni * ov;
      hipLaunchKernelGGL(diag_kernel, dim3(unsigned((nt + 255) / 256)), dim3(256), 0, s, dg, o, v, op, kp, k2, op2,
                         i0, ni, Foo, Fvv, W4T, WW, Bc, t2);
      GFCC_HIP(hipGetLastError());
    }
    GFCC_HIP(hipStreamSynchronize(s));
  }

  // ================================================================= 1h rows
  // sigma_i = -sum_m Foo[m,i] r_m + sum_(mne) U[i,(m,n,e)] r_mne with
  // U = 2 d_im Fov[n,e] - d_in Fov[m,e] - 2 Wooov[m,n,i,e] + Wooov[n,m,i,e]
  {
    double* U = c->Uop.as<double>();
    TView W3 = tview(Wooov, {o, o, o, v});
    permute(tview(Foo, {o, o}), std::array<int, 2>{1, 0}.data(), -1.0, tview_s(U, {o, o}, {Dp, 1}), 0.0, s);
    TView u2v = tview_s(U + op, {o, o, o, v}, {Dp, ov, v, 1});  // [i][m][n][e]
    const int pa[4] = {2, 0, 1, 3}, pb[4] = {2, 1, 0, 3};
    permute(W3, pa, -2.0, u2v, 0.0, s);
    permute(W3, pb, 1.0, u2v, 1.0, s);
    TView fb = tview_s(Fov, {o, o, v}, {0, v, 1});  // broadcast over i
    permute(fb, id3, 2.0, tview_s(U + op, {o, o, v}, {Dp + ov, v, 1}), 1.0, s);  // i = m: [i][n][e]
    permute(fb, id3, -1.0, tview_s(U + op, {o, o, v}, {Dp + v, ov, 1}), 1.0, s);  // i = n: [i][m][e]
  }

  // ================================================================= left vectors c_q (rows of [o][Dp])
  //  c(1h)[q,i]       = d_qi - sum_a l_ia t_qa - sum_jab (2 l_ij^ab - l_ij^ba) t_qj^ab
  //  c(2h1p)[q,k,l,c] = 2 d_qk l_lc - d_ql l_kc - sum_a t_qa (2 l_kl^ac - l_kl^ca)
  {
    const double* l2 = sys->l2 ? sys->l2 : t2;
    if (sys->l2) {  // keep a Lambda2 that differs from t2 (read in place: the caller's buffer)
      DBuf dflag;
      dflag.ensure(sizeof(int), s);
      hipLaunchKernelGGL(differ_kernel, dim3(1024), dim3(256), 0, s, sys->l2, t2, oov * v, dflag.as<int>());
      GFCC_HIP(hipGetLastError());
      int differ = 0;
      GFCC_HIP(hipMemcpyAsync(&differ, dflag.p, sizeof(int), hipMemcpyDeviceToHost, s));
      GFCC_HIP(hipStreamSynchronize(s));
      if (differ) c->l2 = sys->l2;
    }
    double* Cq = c->left.as<double>();
    add_diag(Cq, o, Dp + 1, nullptr, 1.0, 0.0, s);
    TView c1 = tview_s(Cq, {o, o}, {Dp, 1});  // [q][i]
    ein("ia,qa->qi", -1.0, tview(const_cast<double*>(l1), {o, v}), T1, 1.0, c1, scr, s);
    // -2 sum_(jab) l2[i,(jab)] t2[q,(jab)] -> C[i][q] at Cq[q][i]
    g64(mk(l2, lin(o * vv), t2, lin(o * vv), Cq, lin(1), lin(Dp), o, o, o * vv, -2.0, 1.0), scr, s);
    // + sum_(jab) l2[i,j,b,a] t2[q,j,a,b]: chunks of j with t2[q,j,b,a] laid out as [q][(j,a,b)]
    {
      const int64_t cj = clamp_chunk(avail, double(o * vv) * 8.0, o);
      DBuf b_t;
      b_t.ensure(size_t(o * cj * vv) * 8, s);
      double* Ts = b_t.as<double>();
      for (int64_t j0 = 0; j0 < o; j0 += cj) {
        const int64_t nj = std::min(cj, o - j0);
        permute(tview_s(const_cast<double*>(t2) + j0 * vv, {o, nj, v, v}, {o * vv, vv, 1, v}), id4, 1.0,
                tview_s(Ts, {o, nj, v, v}, {nj * vv, vv, v, 1}), 0.0, s);
        g64(mk(l2 + j0 * vv, lin(o * vv), Ts, lin(nj * vv), Cq, lin(1), lin(Dp), o, o, nj * vv, 1.0, 1.0), scr, s);
      }
      GFCC_HIP(hipStreamSynchronize(s));
    }
    const double* l1p = l1;
    TView lb = tview_s(const_cast<double*>(l1p), {o, o, v}, {0, v, 1});
    permute(lb, id3, 2.0, tview_s(Cq + op, {o, o, v}, {Dp + ov, v, 1}), 1.0, s);   // q = k: [q][l][c]
    permute(lb, id3, -1.0, tview_s(Cq + op, {o, o, v}, {Dp + v, ov, 1}), 1.0, s);  // q = l: [q][k][c]
    // + sum_a t1[q,a] l2[k,l,c,a]: C[q][(k,l,c)]
    g64(mk(t1, lin(v), l2, lin(v), Cq + op, lin(Dp), lin(1), o, oov, v, 1.0, 1.0), scr, s);
    // - 2 sum_a t1[q,a] l2[k,l,a,c] = -2 sum_a t1[q,a] l2[l,k,c,a]: batched over k, rows (l,c)
    {
      GemmArgs g = mk(t1, lin(v), l2, two(v, o * vv, v), Cq + op, lin(Dp), lin(1), o, ov, v, -2.0, 1.0);
      g.batch = int(o);
      g.bz = lin(vv);
      g.cz = lin(ov);
      g64(g, scr, s);
    }
  }
  // ---- amplitudes for virtual-orbital right-hand sides and left vectors
  GFCC_HIP(hipMemcpyAsync(c->t1c.p, t1, size_t(ov) * 8, hipMemcpyDeviceToDevice, s));
  GFCC_HIP(hipMemcpyAsync(c->l1c.p, l1, size_t(ov) * 8, hipMemcpyDeviceToDevice, s));
  GFCC_HIP(hipStreamSynchronize(s));
  // the contraction engine's staging buffers are build-sized; the solver needs only small
  // split-K partials from them, so give the memory back
  for (auto& b : scr.b) b.release();
}

// Reduced-precision copies of the two-body operands with power-of-two scales.
void build_lowprec(gfcc_ctx* c, int which, hipStream_t s) {
  if (c->sector == 1) {
    GFCC_CHECK(which == 2, GFCC_E_ARG, "the electron-attachment context has FP16 copies only");
    build_ea_lowprec(c, s);
    return;
  }
  GFCC_CHECK(c->sector == 0, GFCC_E_ARG, "the open-shell context has no reduced-precision copies");
  auto& L = c->lp[which];
  if (L.built) return;
  // one reduced-precision set at a time: the others are released (and rebuilt when asked for)
  for (int w = 0; w < 3; ++w) {
    if (w == which || !c->lp[w].built) continue;
    GFCC_HIP(hipStreamSynchronize(s));
    auto& O = c->lp[w];
    for (DBuf* b : {&O.WW, &O.W4T, &O.WovooT, &O.t2, &O.LovC}) b->release();
    O.built = false;
  }
  const Prec p = which == 0 ? Prec::F32 : (which == 1 ? Prec::BF16 : Prec::F16);
  const int64_t esz = which == 0 ? 4 : 2;
  auto mk_copy = [&](DBuf& dst, const double* src, int64_t n, double& scale) {
    const double am = amax_host(src, n, s, c->scr);
    scale = (am > 0.0) ? std::ldexp(1.0, -std::ilogb(am)) : 1.0;  // amax -> [1, 2)
    dst.ensure(size_t(n * esz), s);
    convert_f64(src, dst.p, p, n, scale, s);
  };
  mk_copy(L.WW, c->WW.as<double>(), c->ov * c->k2, L.sWW);
  mk_copy(L.W4T, c->W4T.as<double>(), c->oo * c->op2, L.sW4T);
  mk_copy(L.WovooT, c->WovooT.as<double>(), c->oov * c->o_pad, L.sWovooT);
  mk_copy(L.t2, c->t2, c->oov * c->v, L.st2);
  mk_copy(L.LovC, c->LovC.as<double>(), c->Q * c->kp, L.sLovC);
  GFCC_HIP(hipStreamSynchronize(s));
  L.built = true;
}

}  // namespace gfcc

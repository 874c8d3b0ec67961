// The open-shell (spin-unrestricted) IP term of the GFCCSD Green's function.
//
// Paper, Theory section (the retarded IP term) for a reference with different numbers of alpha
// and beta electrons, as in the open-shell GFCCSD-IP of the Evaluation section (Table 2): every
// quantity is written over spin orbitals, so one set of equations covers both ionised sectors
// (an alpha or a beta electron removed).
//
// Spin orbitals: occupied [alpha 0..oa-1, beta 0..ob-1], then virtual [alpha oa..n-1,
// beta ob..n-1]; o = oa + ob, v = va + vb.  Vectors: r_i on [0, o), r_ij^a at (i*o + j)*v + a
// of the second block with both orders of the hole pair stored (r_ji^a = -r_ij^a), i.e.
// R = sum_i r_i a_i + 1/2 sum_ija r_ij^a a_a^+ a_j a_i.  The left rows carry 1/2 on their 2h1p
// block so that a plain dot product counts each pair once.
//
// The inputs come in spin blocks; the build assembles spin-orbital Cholesky vectors
// L_so[Q][P][R] = d(s_P, s_R) L_s[Q][p][r] (block diagonal in spin), so that
// <pq|rs> = sum_Q L_so[Q][p][r] L_so[Q][q][s] carries the spin deltas by itself, and the
// amplitudes as antisymmetric spin-orbital tensors.  The Hbar blocks and the sigma product
// are FP64 contractions on MFMA (the contraction engine).
//
//   sigma_i    = -Foo[m,i] r_m + Fov[m,e] r_im^e - 1/2 Wooov[m,n,i,e] r_mn^e
//   sigma_ij^a = -Wovoo[m,a,i,j] r_m + Fvv[a,e] r_ij^e - Foo[m,i] r_mj^a + Foo[m,j] r_mi^a
//                + 1/2 Woooo[m,n,i,j] r_mn^a + Wovvo[m,a,e,j] r_im^e - Wovvo[m,a,e,i] r_jm^e
//                + Z_e t_ij^ae,   Z_e = 1/2 <mn||ef> r_mn^f          (sums over repeated indices)
#include <cmath>

#include "ctx.h"

namespace gfcc {
namespace {

unsigned nblk(int64_t n) { return unsigned(std::min<int64_t>((n + 255) / 256, 65535)); }

struct SpinMap {
  int64_t n, oa, ob, o, v;
  __host__ __device__ int spin_occ(int64_t i) const { return i < oa ? 0 : 1; }
  __host__ __device__ int64_t spat_occ(int64_t i) const { return i < oa ? i : i - oa; }
  __host__ __device__ int spin_vir(int64_t a) const { return a < n - oa ? 0 : 1; }
  // virtual index inside its spin block (0-based among that spin's virtuals)
  __host__ __device__ int64_t vrel(int64_t a) const { return a < n - oa ? a : a - (n - oa); }
  // spatial orbital of spin orbital k of the combined list (occupied then virtual)
  __host__ __device__ void orb(int64_t k, int& s, int64_t& p) const {
    if (k < o) {
      s = spin_occ(k);
      p = spat_occ(k);
    } else {
      const int64_t a = k - o;
      s = spin_vir(a);
      p = (s == 0 ? oa : ob) + vrel(a);
    }
  }
};

// L_so[Q][k][m] = d(s_k, s_m) L_s[Q][p_k][p_m]
__global__ void lso_kernel(SpinMap M, const double* __restrict__ La, const double* __restrict__ Lb,
                           double* __restrict__ L, int64_t Q) {
  const int64_t N = M.o + M.v, n = M.n;
  const int64_t total = Q * N * N;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += int64_t(gridDim.x) * blockDim.x) {
    const int64_t m = t % N, k = (t / N) % N, q = t / (N * N);
    int sk, sm;
    int64_t pk, pm;
    M.orb(k, sk, pk);
    M.orb(m, sm, pm);
    double val = 0.0;
    if (sk == sm) val = (sk == 0 ? La : Lb)[(q * n + pk) * n + pm];
    L[t] = val;
  }
}

// spin-orbital amplitudes from the blocks: t1 [o][v], t2 [o][o][v][v] antisymmetric
__global__ void amp1_kernel(SpinMap M, const double* __restrict__ a1, const double* __restrict__ b1,
                            double* __restrict__ t1) {
  const int64_t total = M.o * M.v;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += int64_t(gridDim.x) * blockDim.x) {
    const int64_t i = t / M.v, a = t % M.v;
    const int si = M.spin_occ(i), sa = M.spin_vir(a);
    double val = 0.0;
    if (si == sa) val = si == 0 ? a1[M.spat_occ(i) * (M.n - M.oa) + M.vrel(a)]
                                : b1[M.spat_occ(i) * (M.n - M.ob) + M.vrel(a)];
    t1[t] = val;
  }
}

__global__ void amp2_kernel(SpinMap M, const double* __restrict__ aa, const double* __restrict__ ab,
                            const double* __restrict__ bb, double* __restrict__ t2) {
  const int64_t o = M.o, v = M.v, va = M.n - M.oa, vb = M.n - M.ob;
  const int64_t total = o * o * v * v;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += int64_t(gridDim.x) * blockDim.x) {
    const int64_t b = t % v, a = (t / v) % v, j = (t / (v * v)) % o, i = t / (v * v * o);
    const int si = M.spin_occ(i), sj = M.spin_occ(j), sa = M.spin_vir(a), sb = M.spin_vir(b);
    const int64_t pi = M.spat_occ(i), pj = M.spat_occ(j), ra = M.vrel(a), rb = M.vrel(b);
    double val = 0.0;
    if (si == sj) {
      if (sa == si && sb == si)
        val = si == 0 ? aa[((pi * M.oa + pj) * va + ra) * va + rb] : bb[((pi * M.ob + pj) * vb + ra) * vb + rb];
    } else if (si == 0) {  // i alpha, j beta: t_{i a, j b} with (a alpha, b beta) or swapped
      if (sa == 0 && sb == 1) val = ab[((pi * M.ob + pj) * va + ra) * vb + rb];
      else if (sa == 1 && sb == 0) val = -ab[((pi * M.ob + pj) * va + rb) * vb + ra];
    } else {  // i beta, j alpha
      if (sa == 0 && sb == 1) val = -ab[((pj * M.ob + pi) * va + ra) * vb + rb];
      else if (sa == 1 && sb == 0) val = ab[((pj * M.ob + pi) * va + rb) * vb + ra];
    }
    t2[t] = val;
  }
}

__global__ void diag_eps_kernel(double* __restrict__ F, const double* __restrict__ eps, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) F[i * n + i] += eps[i];
}

// eps_so[k] for the combined list
__global__ void eps_so_kernel(SpinMap M, const double* __restrict__ ea, const double* __restrict__ eb,
                              double* __restrict__ e) {
  const int64_t N = M.o + M.v;
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= N) return;
  int s;
  int64_t p;
  M.orb(k, s, p);
  e[k] = (s == 0 ? ea : eb)[p];
}

// tau = t2 + t1 t1 - t1 t1 (antisymmetrised)
__global__ void tau_so_kernel(const double* __restrict__ t2, const double* __restrict__ t1, double* __restrict__ tau,
                              int64_t o, int64_t v) {
  const int64_t total = o * o * v * v;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += int64_t(gridDim.x) * blockDim.x) {
    const int64_t b = t % v, a = (t / v) % v, j = (t / (v * v)) % o, i = t / (v * v * o);
    tau[t] = t2[t] + t1[i * v + a] * t1[j * v + b] - t1[i * v + b] * t1[j * v + a];
  }
}

// exact diagonal over the unique basis, stored at both (i,j) and (j,i); padding 1.0
__global__ void uhf_diag_kernel(double* __restrict__ dg, const double* __restrict__ Foo,
                                const double* __restrict__ Fvv, const double* __restrict__ W4,
                                const double* __restrict__ Wvo, const double* __restrict__ oovv,
                                const double* __restrict__ t2, int64_t o, int64_t v, int64_t p1, int64_t Dp) {
  const int64_t n2 = o * o * v;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < Dp; t += int64_t(gridDim.x) * blockDim.x) {
    double d = 1.0;
    if (t < o) {
      d = -Foo[t * o + t];
    } else if (t >= p1 && t - p1 < n2) {
      const int64_t idx = t - p1, a = idx % v, j = (idx / v) % o, i = idx / (v * o);
      d = Fvv[a * v + a] - Foo[i * o + i] - Foo[j * o + j] + W4[((i * o + j) * o + i) * o + j] +
          Wvo[((j * v + a) * v + a) * o + j] + Wvo[((i * v + a) * v + a) * o + i];
      double tb = 0.0;
      for (int64_t e = 0; e < v; ++e) tb += oovv[((i * o + j) * v + e) * v + a] * t2[((i * o + j) * v + a) * v + e];
      d += tb;
    }
    dg[t] = d;
  }
}

// right-hand sides: occupied p -> e_p; virtual p = o + a -> r_i = t1[i,a], r_ij^b = t2[i,j,a,b]
__global__ void uhf_rhs_kernel(const int64_t* __restrict__ orb, const double* __restrict__ t1,
                               const double* __restrict__ t2, double* __restrict__ out, int64_t o, int64_t v,
                               int64_t p1, int64_t Dp) {
  const int64_t r = blockIdx.y, p = orb[r];
  double* row = out + r * Dp;
  const int64_t n2 = o * o * v;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < Dp; t += int64_t(gridDim.x) * blockDim.x) {
    double val = 0.0;
    if (p < o) {
      val = (t == p) ? 1.0 : 0.0;
    } else {
      const int64_t a = p - o;
      if (t < o) {
        val = t1[t * v + a];
      } else if (t >= p1 && t - p1 < n2) {
        const int64_t idx = t - p1, b = idx % v, ij = idx / v;
        val = t2[(ij * v + a) * v + b];
      }
    }
    row[t] = val;
  }
}

// left rows (1/2 on the 2h1p block); S[i][q] = sum_e l1[i,e] t1[q,e] + 1/2 sum_jef l2[i,j,e,f] t2[q,j,e,f]
//   occupied q:  c_i = d_qi - S[i][q];   c_ij^b = d_qi l1[j,b] - d_qj l1[i,b] - sum_e t1[q,e] l2[i,j,e,b]
//   virtual q = o + a:  c_i = l1[i,a];   c_ij^b = l2[i,j,a,b]
__global__ void uhf_left_kernel(const int64_t* __restrict__ orb, const double* __restrict__ t1,
                                const double* __restrict__ l1, const double* __restrict__ l2,
                                const double* __restrict__ S, double* __restrict__ out, int64_t o, int64_t v,
                                int64_t p1, int64_t Dp) {
  const int64_t r = blockIdx.y, q = orb[r];
  double* row = out + r * Dp;
  const int64_t n2 = o * o * v;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < Dp; t += int64_t(gridDim.x) * blockDim.x) {
    double val = 0.0;
    if (t < o) {
      const int64_t i = t;
      if (q < o)
        val = (i == q ? 1.0 : 0.0) - S[i * o + q];
      else
        val = l1[i * v + (q - o)];
    } else if (t >= p1 && t - p1 < n2) {
      const int64_t idx = t - p1, b = idx % v, j = (idx / v) % o, i = idx / (v * o);
      double c;
      if (q < o) {
        c = 0.0;
        if (i == q) c += l1[j * v + b];
        if (j == q) c -= l1[i * v + b];
        for (int64_t e = 0; e < v; ++e) c -= t1[q * v + e] * l2[((i * o + j) * v + e) * v + b];
      } else {
        c = l2[((i * o + j) * v + (q - o)) * v + b];
      }
      val = 0.5 * c;
    }
    row[t] = val;
  }
}

__global__ void zero_pads_kernel(double* __restrict__ y, int64_t n1, int64_t p1, int64_t n2, int64_t Dp) {
  double* yp = y + int64_t(blockIdx.y) * Dp;
  const int64_t w1 = p1 - n1, w2 = Dp - p1 - n2;
  for (int64_t t = threadIdx.x; t < w1 + w2; t += blockDim.x) yp[t < w1 ? n1 + t : p1 + n2 + (t - w1)] = 0.0;
}

}  // namespace

// ------------------------------------------------------------------ build

void build_uhf(gfcc_ctx* c, const gfcc_uhf_system* sys, hipStream_t s) {
  const int64_t n = sys->n, oa = sys->n_occ_a, ob = sys->n_occ_b, Q = sys->n_chol;
  const int64_t o = c->o, v = c->v, N = o + v;
  SpinMap M{n, oa, ob, o, v};
  Scratch& scr = c->scr;
  auto g64 = [&](DBuf& b, int64_t nd) {
    b.ensure(size_t(nd) * 8, s);
    return b.as<double>();
  };
  // spin-orbital inputs
  DBuf b_L, b_eps, b_tau, b_g;
  double* L = g64(b_L, Q * N * N);
  hipLaunchKernelGGL(lso_kernel, dim3(nblk(Q * N * N)), dim3(256), 0, s, M, sys->La, sys->Lb, L, Q);
  double* eps = g64(b_eps, N);
  hipLaunchKernelGGL(eps_so_kernel, dim3(nblk(N)), dim3(256), 0, s, M, sys->eps_a, sys->eps_b, eps);
  double* t1 = g64(c->uhf.t1, o * v);
  double* t2 = g64(c->uhf.t2, o * o * v * v);
  hipLaunchKernelGGL(amp1_kernel, dim3(nblk(o * v)), dim3(256), 0, s, M, sys->t1a, sys->t1b, t1);
  hipLaunchKernelGGL(amp2_kernel, dim3(nblk(o * o * v * v)), dim3(256), 0, s, M, sys->t2aa, sys->t2ab, sys->t2bb, t2);
  const bool lam = sys->l1a != nullptr;
  double* l1 = g64(c->uhf.l1, o * v);
  double* l2 = g64(c->uhf.l2, o * o * v * v);
  if (lam) {
    hipLaunchKernelGGL(amp1_kernel, dim3(nblk(o * v)), dim3(256), 0, s, M, sys->l1a, sys->l1b, l1);
    hipLaunchKernelGGL(amp2_kernel, dim3(nblk(o * o * v * v)), dim3(256), 0, s, M, sys->l2aa, sys->l2ab, sys->l2bb,
                       l2);
  } else {
    GFCC_HIP(hipMemcpyAsync(l1, t1, size_t(o * v) * 8, hipMemcpyDeviceToDevice, s));
    GFCC_HIP(hipMemcpyAsync(l2, t2, size_t(o * o * v * v) * 8, hipMemcpyDeviceToDevice, s));
  }
  double* tau = g64(b_tau, o * o * v * v);
  hipLaunchKernelGGL(tau_so_kernel, dim3(nblk(o * o * v * v)), dim3(256), 0, s, t2, t1, tau, o, v);
  GFCC_HIP(hipGetLastError());

  // <pq||rs> blocks: <pq|rs> = sum_Q L[Q,p,r] L[Q,q,s]
  auto Lb = [&](int64_t r0, int64_t nr, int64_t c0, int64_t nc) {
    return tview_s(L + r0 * N + c0, {Q, nr, nc}, {N * N, N, 1});
  };
  const int64_t O0 = 0, V0 = o;
  struct Blk {
    int64_t s0, n0;
  };
  auto anti = [&](DBuf& buf, Blk P, Blk Qb, Blk R, Blk S) {
    double* p = g64(buf, P.n0 * Qb.n0 * R.n0 * S.n0);
    TView out = tview(p, {P.n0, Qb.n0, R.n0, S.n0});
    ein("Xpr,Xqs->pqrs", 1.0, Lb(P.s0, P.n0, R.s0, R.n0), Lb(Qb.s0, Qb.n0, S.s0, S.n0), 0.0, out, scr, s);
    ein("Xps,Xqr->pqrs", -1.0, Lb(P.s0, P.n0, S.s0, S.n0), Lb(Qb.s0, Qb.n0, R.s0, R.n0), 1.0, out, scr, s);
    return out;
  };
  const Blk bo{O0, o}, bv{V0, v};
  DBuf b_oooo, b_ooov, b_oovo, b_ovvo, b_ovvv, b_vovv, b_ovoo;
  const TView oooo = anti(b_oooo, bo, bo, bo, bo);
  const TView ooov = anti(b_ooov, bo, bo, bo, bv);
  const TView oovo = anti(b_oovo, bo, bo, bv, bo);
  const TView oovv = anti(c->uhf.oovv, bo, bo, bv, bv);
  const TView ovvo = anti(b_ovvo, bo, bv, bv, bo);
  const TView ovvv = anti(b_ovvv, bo, bv, bv, bv);
  const TView vovv = anti(b_vovv, bv, bo, bv, bv);
  const TView ovoo = anti(b_ovoo, bo, bv, bo, bo);
  const TView T1 = tview(t1, {o, v});
  const TView T2 = tview(t2, {o, o, v, v});
  const TView TAU = tview(tau, {o, o, v, v});

  // one-body blocks
  const TView Fov = tview(g64(c->Fov, o * v), {o, v});
  const TView Foo = tview(g64(c->Foo, o * o), {o, o});
  const TView Fvv = tview(g64(c->Fvv, v * v), {v, v});
  ein("nf,mnef->me", 1.0, T1, oovv, 0.0, Fov, scr, s);
  GFCC_HIP(hipMemsetAsync(Foo.p, 0, size_t(o * o) * 8, s));
  GFCC_HIP(hipMemsetAsync(Fvv.p, 0, size_t(v * v) * 8, s));
  hipLaunchKernelGGL(diag_eps_kernel, dim3(nblk(o)), dim3(256), 0, s, Foo.p, eps, o);
  hipLaunchKernelGGL(diag_eps_kernel, dim3(nblk(v)), dim3(256), 0, s, Fvv.p, eps + o, v);
  GFCC_HIP(hipGetLastError());
  ein("ie,me->mi", 1.0, T1, Fov, 1.0, Foo, scr, s);
  ein("ne,mnie->mi", 1.0, T1, ooov, 1.0, Foo, scr, s);
  ein("inef,mnef->mi", 0.5, T2, oovv, 1.0, Foo, scr, s);
  ein("ma,me->ae", -1.0, T1, Fov, 1.0, Fvv, scr, s);
  ein("mf,amef->ae", 1.0, T1, vovv, 1.0, Fvv, scr, s);
  ein("mnaf,mnef->ae", -0.5, T2, oovv, 1.0, Fvv, scr, s);

  // two-body blocks
  const int id4[4] = {0, 1, 2, 3};
  const TView W4 = tview(g64(c->uhf.Woooo, o * o * o * o), {o, o, o, o});
  permute(oooo, id4, 1.0, W4, 0.0, s);
  ein("je,mnie->mnij", 1.0, T1, ooov, 1.0, W4, scr, s);
  ein("ie,mnje->mnij", -1.0, T1, ooov, 1.0, W4, scr, s);
  ein("ijef,mnef->mnij", 0.5, TAU, oovv, 1.0, W4, scr, s);
  const TView W3 = tview(g64(c->uhf.Wooov, o * o * o * v), {o, o, o, v});
  permute(ooov, id4, 1.0, W3, 0.0, s);
  ein("if,mnfe->mnie", 1.0, T1, oovv, 1.0, W3, scr, s);
  const TView Wvo = tview(g64(c->uhf.Wovvo, o * v * v * o), {o, v, v, o});
  permute(ovvo, id4, 1.0, Wvo, 0.0, s);
  ein("jf,mbef->mbej", 1.0, T1, ovvv, 1.0, Wvo, scr, s);
  ein("nb,mnej->mbej", -1.0, T1, oovo, 1.0, Wvo, scr, s);
  ein("jnfb,mnef->mbej", -1.0, T2, oovv, 1.0, Wvo, scr, s);
  {
    DBuf b_h;  // H[m,n,e,j] = sum_f t_jf <mn||ef>
    const TView H = tview(g64(b_h, o * o * v * o), {o, o, v, o});
    ein("jf,mnef->mnej", 1.0, T1, oovv, 0.0, H, scr, s);
    ein("nb,mnej->mbej", -1.0, T1, H, 1.0, Wvo, scr, s);
  }
  const TView Wovoo = tview(g64(c->uhf.Wovoo, o * v * o * o), {o, v, o, o});
  {
    permute(ovoo, id4, 1.0, Wovoo, 0.0, s);
    ein("me,ijbe->mbij", -1.0, Fov, T2, 1.0, Wovoo, scr, s);
    ein("nb,mnij->mbij", -1.0, T1, W4, 1.0, Wovoo, scr, s);
    ein("mbef,ijef->mbij", 0.5, ovvv, TAU, 1.0, Wovoo, scr, s);
    ein("mnie,jnbe->mbij", 1.0, ooov, T2, 1.0, Wovoo, scr, s);
    ein("mnje,inbe->mbij", -1.0, ooov, T2, 1.0, Wovoo, scr, s);
    DBuf b_y;  // Y[m,b,e,j] = <mb||ej> - sum_nf t_nj^bf <mn||ef>
    const TView Y = tview(g64(b_y, o * v * v * o), {o, v, v, o});
    permute(ovvo, id4, 1.0, Y, 0.0, s);
    ein("njbf,mnef->mbej", -1.0, T2, oovv, 1.0, Y, scr, s);
    ein("ie,mbej->mbij", 1.0, T1, Y, 1.0, Wovoo, scr, s);
    ein("je,mbei->mbij", -1.0, T1, Y, 1.0, Wovoo, scr, s);
  }
  // left-vector helper S[i][q]
  {
    const TView S = tview(g64(c->uhf.S, o * o), {o, o});
    ein("ie,qe->iq", 1.0, tview(l1, {o, v}), T1, 0.0, S, scr, s);
    ein("ijef,qjef->iq", 0.5, tview(l2, {o, o, v, v}), T2, 1.0, S, scr, s);
  }
  double* dg = g64(c->diag, c->Dp);
  hipLaunchKernelGGL(uhf_diag_kernel, dim3(nblk(c->Dp)), dim3(256), 0, s, dg, Foo.p, Fvv.p, W4.p, Wvo.p, oovv.p, t2,
                     o, v, c->p1, c->Dp);
  GFCC_HIP(hipGetLastError());
  GFCC_HIP(hipStreamSynchronize(s));  // build temporaries are released on return
}

// ------------------------------------------------------------------ sigma

void uhf_sigma_planes(gfcc_ctx* c, int64_t P, const double* x, double* y, hipStream_t s) {
  if (P <= 0) return;
  const int64_t o = c->o, v = c->v, Dp = c->Dp, p1 = c->p1;
  Scratch& scr = c->scr;
  double* xp = const_cast<double*>(x);
  const TView r1 = tview_s(xp, {P, o}, {Dp, 1});
  const TView r2 = tview_s(xp + p1, {P, o, o, v}, {Dp, o * v, v, 1});
  const TView s1 = tview_s(y, {P, o}, {Dp, 1});
  const TView s2 = tview_s(y + p1, {P, o, o, v}, {Dp, o * v, v, 1});
  const TView Foo = tview(c->Foo.as<double>(), {o, o});
  const TView Fov = tview(c->Fov.as<double>(), {o, v});
  const TView Fvv = tview(c->Fvv.as<double>(), {v, v});
  const TView W4 = tview(c->uhf.Woooo.as<double>(), {o, o, o, o});
  const TView W3 = tview(c->uhf.Wooov.as<double>(), {o, o, o, v});
  const TView Wvo = tview(c->uhf.Wovvo.as<double>(), {o, v, v, o});
  const TView Wovoo = tview(c->uhf.Wovoo.as<double>(), {o, v, o, o});
  const TView oovv = tview(c->uhf.oovv.as<double>(), {o, o, v, v});
  const TView T2 = tview(c->uhf.t2.as<double>(), {o, o, v, v});
  c->uhf.ws_z.ensure(size_t(P * v) * 8, s);
  const TView Z = tview(c->uhf.ws_z.as<double>(), {P, v});
  prof_begin(c, "uhf_sigma", s);
  ein("mi,xm->xi", -1.0, Foo, r1, 0.0, s1, scr, s);
  ein("me,xime->xi", 1.0, Fov, r2, 1.0, s1, scr, s);
  ein("mnie,xmne->xi", -0.5, W3, r2, 1.0, s1, scr, s);
  ein("maij,xm->xija", -1.0, Wovoo, r1, 0.0, s2, scr, s);
  ein("ae,xije->xija", 1.0, Fvv, r2, 1.0, s2, scr, s);
  ein("mi,xmja->xija", -1.0, Foo, r2, 1.0, s2, scr, s);
  ein("mj,xmia->xija", 1.0, Foo, r2, 1.0, s2, scr, s);
  ein("mnij,xmna->xija", 0.5, W4, r2, 1.0, s2, scr, s);
  ein("maej,xime->xija", 1.0, Wvo, r2, 1.0, s2, scr, s);
  ein("maei,xjme->xija", -1.0, Wvo, r2, 1.0, s2, scr, s);
  ein("mnef,xmnf->xe", 0.5, oovv, r2, 0.0, Z, scr, s);
  ein("xe,ijae->xija", 1.0, Z, T2, 1.0, s2, scr, s);
  hipLaunchKernelGGL(zero_pads_kernel, dim3(1, unsigned(P)), dim3(256), 0, s, y, c->n1, p1, c->n2, Dp);
  GFCC_HIP(hipGetLastError());
  prof_end(c, "uhf_sigma", s, 0.0, 0.0);
}

void uhf_rhs_rows(gfcc_ctx* c, int64_t n, const int64_t* orb_dev, double* out, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(uhf_rhs_kernel, dim3(nblk(c->Dp), unsigned(n)), dim3(256), 0, s, orb_dev,
                     c->uhf.t1.as<double>(), c->uhf.t2.as<double>(), out, c->o, c->v, c->p1, c->Dp);
  GFCC_HIP(hipGetLastError());
}

void uhf_left_rows(gfcc_ctx* c, int64_t n, const int64_t* orb_dev, double* out, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(uhf_left_kernel, dim3(nblk(c->Dp), unsigned(n)), dim3(256), 0, s, orb_dev,
                     c->uhf.t1.as<double>(), c->uhf.l1.as<double>(), c->uhf.l2.as<double>(), c->uhf.S.as<double>(),
                     out, c->o, c->v, c->p1, c->Dp);
  GFCC_HIP(hipGetLastError());
}

}  // namespace gfcc

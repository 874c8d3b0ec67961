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
// The ring terms are the hot spot (12 o^3 v^2 flops per complex vector), two GEMMs
// against the ring matrix WW[(j,a)] = [Wovvo | Wovov] (one-body terms folded in):
//   P1: s2[(p,i)][(j,a)] += [2R - RT | -R][(p,i)] . WW[(j,a)]^T    (K = 2 o v)
//       (2 Wovvo - Wovov) R - Wovvo RT = Wovvo (2R - RT) - Wovov R,  R[(p,i)][(m,e)] = r2[i][m][e],
//       RT[(p,i)][(m,e)] = r2[m][i][e]
//   P2: s2[(p,j)][(i,a)] -= RT[(p,j)] . Wovov[(i,a)]^T                 (scattered store)
// The three-body z goes through the Cholesky vectors: with
//   U[(p,m)][Q] = sum_(n,f) (2R - RT)[(p,m)][(n,f)] L[Q][n][o+f]   (the first half of P1's operand)
//   z[p][e]     = sum_(m,Q) U[(p,m)][Q] L[Q][m][o+e]
// and s2[p][(i,j,a)] -= sum_e z[p][e] t2[j][i][a][e] (t_ij^ea = t_ji^ae) reads the
// caller's t2 in place, one occupied i per batch.
// In FP32/BF16 mode the ring, ladder, U, three-body and 2h1p <- 1h products read
// reduced-precision copies; the one-body diagonal, z and the 1h rows stay FP64.
#include <algorithm>
#include <cstring>
#include <string>

#include "ctx.h"

namespace gfcc {

template <typename T> __device__ __forceinline__ T cvt(double x);
template <> __device__ __forceinline__ double cvt<double>(double x) { return x; }
template <> __device__ __forceinline__ float cvt<float>(double x) { return float(x); }
template <> __device__ __forceinline__ __bf16 cvt<__bf16>(double x) { return __bf16(float(x)); }
template <> __device__ __forceinline__ _Float16 cvt<_Float16>(double x) { return _Float16(float(x)); }

// Scale of the vector operands of the FP16 products (FP16 has five exponent bits): the
// power of two that maps the largest magnitude of the P input planes into [1, 2).  Partial
// maxima per block, then one block turns them into sc[0] = s and sc[1] = 1/s.  A zero or
// non-finite maximum gives s = 1 (a non-finite vector then stays non-finite for the solver).
__global__ void amax_part_kernel(const double* __restrict__ x, int64_t n, double* __restrict__ part) {
  __shared__ double red[256];
  double m = 0.0;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n; t += int64_t(gridDim.x) * blockDim.x)
    m = fmax(m, fabs(x[t]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}
// which = 0: sc[0] = s, sc[1] = 1/s from the planes;  which = 1: sc[2] = s_z, sc[3] = 1/(s s_z) from z
__global__ void scale_final_kernel(const double* __restrict__ part, int n, double* __restrict__ sc, int which) {
  __shared__ double red[256];
  double m = 0.0;
  for (int t = threadIdx.x; t < n; t += blockDim.x) m = fmax(m, part[t]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double am = red[0];
    const double sv = (am > 0.0 && am <= 1.0e300) ? ldexp(1.0, -ilogb(am)) : 1.0;
    if (which == 0) {
      sc[0] = sv;
      sc[1] = 1.0 / sv;
    } else {
      sc[2] = sv;
      sc[3] = 1.0 / (sc[0] * sv);
    }
  }
}

// Per plane p and element t = (i, m, e) of the 2h1p block:
//   A1[(p,i)][(m,e)] = 2 r[i][m][e] - r[m][i][e],  A1[(p,i)][kp + (m,e)] = -r[i][m][e]  (row stride k2)
//   RT[(p,i)][(m,e)] = r[m][i][e]                                                      (row stride kp)
//   y2[p][t] = d1b[t] x2[p][t]   (FP64 diagonal one-body part; initialises y2)
// and r1l[p][m] = r1[p][m] (reduced-precision copy of the 1h part, row stride o_pad).
template <typename T>
__global__ void make_ops_kernel(const double* __restrict__ x, T* __restrict__ A1, T* __restrict__ RT,
                                T* __restrict__ r1l, double* __restrict__ y, const double* __restrict__ d1b, int64_t o,
                                int64_t v, int64_t Dp, int64_t o_pad, int64_t kp, int64_t k2,
                                const double* __restrict__ vsc) {
  const int64_t oov = o * o * v, ov = o * v;
  const int64_t p = blockIdx.y;
  const double* xp = x + p * Dp + o_pad;
  double* yp = y + p * Dp + o_pad;
  const double sv = vsc ? vsc[0] : 1.0;  // operand scale of the FP16 form (1 otherwise)
  const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r1l && gid < o) r1l[p * o_pad + gid] = cvt<T>(sv * x[p * Dp + gid]);
  for (int64_t t = gid; t < oov; t += int64_t(gridDim.x) * blockDim.x) {
    const int64_t e = t % v, m = (t / v) % o, i = t / ov;
    const int64_t me = m * v + e;
    const double r = xp[t];
    const double rt = xp[m * ov + i * v + e];
    T* a = A1 + (p * o + i) * k2;
    a[me] = cvt<T>(sv * (2.0 * r - rt));
    a[kp + me] = cvt<T>(-sv * r);
    RT[(p * o + i) * kp + me] = cvt<T>(sv * rt);
    yp[t] = d1b[t] * r;
  }
  // padding columns of both halves: the products read them (K = kp, 2 kp), and the buffer
  // is shared with copies in other precisions, so stale bytes must not stay there
  const int64_t pad = kp - ov;
  for (int64_t t = gid; t < o * pad; t += int64_t(gridDim.x) * blockDim.x) {
    T* a = A1 + (p * o + t / pad) * k2 + ov + t % pad;
    a[0] = cvt<T>(0.0);
    a[kp] = cvt<T>(0.0);
  }
}

// Ra[p][a][(m,n)] = x[p*Dp + o_pad + (m,n)*v + a]  (row stride op2), LDS-tiled transpose
template <typename T>
__global__ void make_ra_kernel(const double* __restrict__ x, T* __restrict__ Ra, int64_t oo, int64_t v,
                               int64_t Dp, int64_t o_pad, int64_t op2, const double* __restrict__ vsc) {
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
    if (a < v && r < oo) Ra[(p * v + a) * op2 + r] = cvt<T>((vsc ? vsc[0] : 1.0) * tile[threadIdx.x][k]);
  }
}

template <typename T>
__global__ void to_prec_kernel(const double* __restrict__ src, T* __restrict__ dst, int64_t n,
                               const double* __restrict__ sc) {
  const double sv = sc ? *sc : 1.0;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n; t += int64_t(gridDim.x) * blockDim.x)
    dst[t] = cvt<T>(sv * src[t]);
}

static unsigned blocks_for(int64_t n) {
  return unsigned(std::min<int64_t>(std::max<int64_t>((n + 255) / 256, 1), 4096));
}

template <typename T>
static void make_operands(gfcc_ctx* c, int64_t P, const double* x, bool lowp, double* y, const double* vsc,
                          hipStream_t s) {
  const int64_t oov = c->oov;
  hipLaunchKernelGGL((make_ops_kernel<T>), dim3(std::min<int64_t>((oov + 255) / 256, 1024), unsigned(P)), dim3(256),
                     0, s, x, c->ws_A1.as<T>(), c->ws_RT.as<T>(), lowp ? c->ws_r1.as<T>() : nullptr, y,
                     c->d1b.as<double>(), c->o, c->v, c->Dp, c->o_pad, c->kp, c->k2, vsc);
  GFCC_HIP(hipGetLastError());
  dim3 g(unsigned((c->oo + 31) / 32), unsigned((c->v + 31) / 32), unsigned(P));
  hipLaunchKernelGGL((make_ra_kernel<T>), g, dim3(32, 8), 0, s, x, c->ws_Ra.as<T>(), c->oo, c->v, c->Dp, c->o_pad,
                     c->op2, vsc);
  GFCC_HIP(hipGetLastError());
}

// the FP16 form's operand scale of n doubles at x into sc[2 which], sc[2 which + 1]
void vector_scale(gfcc_ctx* c, const double* x, int64_t n, int which, hipStream_t s) {
  c->ws_vsc.ensure(8 * 8, s);
  c->ws_vpart.ensure(1024 * 8, s);
  const unsigned nb = unsigned(std::min<int64_t>(std::max<int64_t>((n + 255) / 256, 1), 1024));
  hipLaunchKernelGGL(amax_part_kernel, dim3(nb), dim3(256), 0, s, x, n, c->ws_vpart.as<double>());
  hipLaunchKernelGGL(scale_final_kernel, dim3(1), dim3(256), 0, s, c->ws_vpart.as<double>(), int(nb),
                     c->ws_vsc.as<double>(), which);
  GFCC_HIP(hipGetLastError());
}

// phases of one sigma: operand copies, the two ring GEMMs, everything else
enum : int { PH_OPS = 1, PH_RING = 2, PH_REST = 4, PH_ALL = 7 };

// With ring_out != nullptr the ring phase returns its two GEMMs (and tiles)
// instead of launching them, for a grouped launch over several systems.
static void sigma_impl(gfcc_ctx* c, int64_t P, const double* x, double* y, gfcc_precision prec, hipStream_t s,
                       int phases, GemmArgs* ring_out, int* ring_cfg) {
  if (P <= 0) return;
  const int64_t o = c->o, v = c->v, ov = c->ov, oo = c->oo, oov = c->oov;
  const int64_t Dp = c->Dp, op = c->o_pad, kp = c->kp, k2 = c->k2, Qp = c->Qp, Q = c->Q;
  const bool lowp = prec != GFCC_FP64;
  const int li = (prec == GFCC_BF16_IR) ? 1 : (prec == GFCC_FP16_IR ? 2 : 0);
  const bool f16 = li == 2;
  const Prec rp = !lowp ? Prec::F64 : (li == 1 ? Prec::BF16 : (f16 ? Prec::F16 : Prec::F32));
  const int64_t esz = !lowp ? 8 : (li ? 2 : 4);
  if (lowp) build_lowprec(c, li, s);
  if (f16) {
    c->ws_vsc.ensure(8 * 8, s);
    c->ws_vpart.ensure(1024 * 8, s);
  }
  // FP16: the vector operands are scaled by sc[0] on conversion; products unscale on the GPU
  const double* sc = f16 ? c->ws_vsc.as<double>() : nullptr;
  const double* inv_s = f16 ? sc + 1 : nullptr;
  c->ws_A1.ensure(size_t(P * o * k2 * esz), s);
  c->ws_RT.ensure(size_t(P * o * kp * esz), s);
  c->ws_Ra.ensure(size_t(P * v * c->op2 * esz), s);
  if (lowp) c->ws_r1.ensure(size_t(P * op * esz), s);
  c->ws_U.ensure(size_t(P * o * Qp) * 8, s);
  c->ws_z.ensure(size_t(P * c->vp) * 8, s);
  if (lowp) c->ws_zl.ensure(size_t(P * c->vp * esz), s);

  const bool whole = phases == PH_ALL;
  if (whole) prof_begin(c, "sigma", s);
  if (phases & PH_OPS) {
    switch (rp) {
      case Prec::F64: make_operands<double>(c, P, x, false, y, nullptr, s); break;
      case Prec::F32: make_operands<float>(c, P, x, true, y, nullptr, s); break;
      case Prec::BF16: make_operands<__bf16>(c, P, x, true, y, nullptr, s); break;
      case Prec::F16:
        vector_scale(c, x, P * Dp, 0, s);
        make_operands<_Float16>(c, P, x, true, y, sc, s);
        break;
    }
  }
  const auto& L = c->lp[li];
  const void* WWp = lowp ? L.WW.p : c->WW.p;
  const void* W4T = lowp ? L.W4T.p : c->W4T.p;
  const void* WovooT = lowp ? L.WovooT.p : c->WovooT.p;
  const void* t2p = lowp ? L.t2.p : static_cast<const void*>(c->t2);
  const void* LovC = lowp ? L.LovC.p : c->LovC.p;
  const double sWW = lowp ? 1.0 / L.sWW : 1.0, sW4T = lowp ? 1.0 / L.sW4T : 1.0;
  const double sWovoo = lowp ? 1.0 / L.sWovooT : 1.0, st2 = lowp ? 1.0 / L.st2 : 1.0;
  const double sLovC = lowp ? 1.0 / L.sLovC : 1.0;

  const double ring1 = 2.0 * double(P) * double(o) * double(ov) * double(ov);  // flops of one (m,e) half
  const char* ring_name = !lowp ? "ring_gemm_fp64" : (li == 1 ? "ring_gemm_bf16" : (f16 ? "ring_gemm_fp16" : "ring_gemm_fp32"));
  const double c_rw = 2.0 * double(P) * double(o) * double(ov) * 8.0;  // read + write of the FP64 output

  // ---- ring terms
  if (phases & PH_RING) {
    GemmArgs g;
    // P1: s2[(p,i)][(j,a)] += [2R - RT | -R] . WW^T
    g.A = c->ws_A1.p;
    g.am = lin(k2);
    g.B = WWp;
    g.bm = lin(k2);
    g.M = P * o;
    g.N = ov;
    g.K = k2;
    g.C = y + op;
    g.cm = two(o, Dp, ov);
    g.cn = lin(1);
    g.alpha = sWW;
    g.alpha_dev = inv_s;
    g.beta = 1.0;  // y2 holds the diagonal one-body part
    const int cfg1 = tuned_cfg(c, rp, g.M, g.N, g.K);
    if (ring_out) {
      ring_out[0] = g;
      ring_cfg[0] = cfg1;
    } else {  // a one-group grouped launch: the ring products get kernels of their own in traces
      const std::string by_tile = std::string(ring_name) + ":" + tile_name(cfg1);
      const double fl = 2.0 * ring1, by = double(ov) * 2.0 * ov * esz + double(P) * o * 2.0 * ov * esz + c_rw;
      prof_begin(c, ring_name, s);
      prof_begin(c, by_tile.c_str(), s);
      gemm_grouped(rp, &g, 1, cfg1, s);
      prof_end(c, by_tile.c_str(), s, fl, by);
      prof_end(c, ring_name, s, fl, by);
    }
    // P2: rows (p, j), cols (i, a) -> s2[p][i][j][a]
    GemmArgs h;
    h.A = c->ws_RT.p;
    h.am = lin(kp);
    h.B = static_cast<const char*>(WWp) + kp * esz;
    h.bm = lin(k2);
    h.M = P * o;
    h.N = ov;
    h.K = ov;
    h.C = y + op;
    h.cm = two(o, Dp, v);
    h.cn = two(v, ov, 1);
    h.alpha = -sWW;
    h.alpha_dev = inv_s;
    h.beta = 1.0;
    const int cfg2 = tuned_cfg(c, rp, h.M, h.N, h.K);
    if (ring_out) {
      ring_out[1] = h;
      ring_cfg[1] = cfg2;
    } else {
      const std::string by_tile = std::string(ring_name) + ":" + tile_name(cfg2);
      const double fl = ring1, by = double(ov) * ov * esz + double(P) * o * ov * esz + c_rw;
      prof_begin(c, ring_name, s);
      prof_begin(c, by_tile.c_str(), s);
      gemm_grouped(rp, &h, 1, cfg2, s);
      prof_end(c, by_tile.c_str(), s, fl, by);
      prof_end(c, ring_name, s, fl, by);
    }
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
    g.alpha_dev = inv_s;
    g.beta = 1.0;
    gemm(rp, g, tuned_cfg(c, rp, g.M, g.N, g.K), s);
  }
  // ---- three-body: U = (2R - RT) . LovC^T (inner precision), z = U . LovT^T (FP64)
  {
    GemmArgs g;
    g.A = c->ws_A1.p;
    g.am = lin(k2);
    g.B = LovC;
    g.bm = lin(kp);
    g.M = P * o;
    g.N = Q;
    g.K = kp;
    g.C = c->ws_U.as<double>();
    g.cm = lin(Qp);
    g.cn = lin(1);
    g.alpha = sLovC;
    g.beta = 0.0;
    gemm(rp, g, tuned_cfg(c, rp, g.M, g.N, g.K), s);
    GemmArgs h;
    h.A = c->ws_U.p;
    h.am = lin(o * Qp);
    h.B = c->LovT.p;
    h.bm = lin(o * Qp);
    h.M = P;
    h.N = v;
    h.K = o * Qp;
    h.C = c->ws_z.as<double>();
    h.cm = lin(c->vp);
    h.cn = lin(1);
    h.alpha = 1.0;
    h.beta = 0.0;
    gemm_auto(Prec::F64, h, c->scr, 0, s);
  }
  // ---- three-body second half: s2[p][(i,j,a)] -= sum_e z[p][e] t2[j][i][a][e], batched over i
  {
    const void* zA = c->ws_z.p;
    if (lowp) {
      const int64_t nz = P * c->vp;
      if (f16) {  // z (already carrying sc[0] through U) gets a scale of its own: sc[2]
        vector_scale(c, c->ws_z.as<double>(), nz, 1, s);
        hipLaunchKernelGGL((to_prec_kernel<_Float16>), dim3(blocks_for(nz)), dim3(256), 0, s, c->ws_z.as<double>(),
                           c->ws_zl.as<_Float16>(), nz, sc + 2);
      } else if (li) {
        hipLaunchKernelGGL((to_prec_kernel<__bf16>), dim3(blocks_for(nz)), dim3(256), 0, s, c->ws_z.as<double>(),
                           c->ws_zl.as<__bf16>(), nz, nullptr);
      } else {
        hipLaunchKernelGGL((to_prec_kernel<float>), dim3(blocks_for(nz)), dim3(256), 0, s, c->ws_z.as<double>(),
                           c->ws_zl.as<float>(), nz, nullptr);
      }
      GFCC_HIP(hipGetLastError());
      zA = c->ws_zl.p;
    }
    GemmArgs g;
    g.A = zA;
    g.am = lin(c->vp);
    g.B = t2p;
    g.bm = two(v, o * v * v, v);
    g.M = P;
    g.N = ov;
    g.K = v;
    g.C = y + op;
    g.cm = lin(Dp);
    g.cn = lin(1);
    g.batch = int(o);
    g.bz = lin(v * v);
    g.cz = lin(ov);
    g.alpha = -st2;
    g.alpha_dev = f16 ? sc + 3 : nullptr;  // 1 / (s s_z)
    g.beta = 1.0;
    gemm(rp, g, gemm_default_cfg(g.M, g.N, g.K), s);
  }
  // ---- 2h1p <- 1h: s2[p][(i,j,a)] -= sum_m r1[p][m] Wovoo[m,a,i,j]
  {
    GemmArgs g;
    if (lowp) {
      g.A = c->ws_r1.p;
      g.am = lin(op);
    } else {
      g.A = x;
      g.am = lin(Dp);
    }
    g.B = WovooT;
    g.bm = lin(op);
    g.M = P;
    g.N = oov;
    g.K = o;
    g.C = y + op;
    g.cm = lin(Dp);
    g.cn = lin(1);
    g.alpha = -sWovoo;
    g.alpha_dev = inv_s;
    g.beta = 1.0;
    gemm(rp, g, tuned_cfg(c, rp, g.M, g.N, g.K), s);
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
  const double total_flops = 3.0 * ring1 + 2.0 * double(P) * (double(oo) * oo * v + double(o) * Q * ov +
                                                              double(o) * Q * v + double(oov) * v + double(oov) * o +
                                                              double(Dp) * o);
  if (whole) prof_end(c, "sigma", s, total_flops, 0.0);
}

void sigma_planes(gfcc_ctx* c, int64_t P, const double* x, double* y, gfcc_precision prec, hipStream_t s) {
  if (c->sector == 1) {
    GFCC_CHECK(prec == GFCC_FP64 || prec == GFCC_FP16_IR, GFCC_E_ARG,
               "the electron-attachment sigma runs in FP64 or FP16");
    ea_sigma_planes(c, P, x, y, prec, s);
    return;
  }
  if (c->sector == 2) {
    GFCC_CHECK(prec == GFCC_FP64, GFCC_E_ARG, "the open-shell sigma runs in FP64 only");
    uhf_sigma_planes(c, P, x, y, s);
    return;
  }
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
  const Prec rp = prec == GFCC_FP64 ? Prec::F64
                  : (prec == GFCC_BF16_IR ? Prec::BF16 : (prec == GFCC_FP16_IR ? Prec::F16 : Prec::F32));
  GemmArgs ring[2][MAX_GEMM_GROUPS];
  int ng = 0, cfg[2] = {0, 0};
  double best = -1.0;
  for (int j = 0; j < nj; ++j) {
    const SigmaJob& J = jobs[j];
    if (J.P <= 0) continue;
    sigma_impl(J.c, J.P, J.x, J.y, prec, s, PH_OPS, nullptr, nullptr);
    GemmArgs g2[2];
    int cj[2] = {0, 0};
    sigma_impl(J.c, J.P, J.x, J.y, prec, s, PH_RING, g2, cj);
    for (int t = 0; t < 2; ++t) ring[t][ng] = g2[t];
    const double size = double(g2[0].M) * double(g2[0].N);
    if (size > best) {
      best = size;
      cfg[0] = cj[0];
      cfg[1] = cj[1];
    }
    ++ng;
  }
  for (int t = 0; t < 2; ++t) gemm_grouped(rp, ring[t], ng, cfg[t], s);
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
                     c->D, c->Dp, c->n1, c->p1);
  GFCC_HIP(hipGetLastError());
}

void from_planes(gfcc_ctx* c, int64_t nb, const double* planes, double* xi, hipStream_t s) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(from_planes_kernel, dim3(blocks_for(c->D), unsigned(nb)), dim3(256), 0, s, planes, xi, nb,
                     c->D, c->Dp, c->n1, c->p1);
  GFCC_HIP(hipGetLastError());
}

// Right-hand sides b_p = abar_p|Phi> on the 1h + 2h1p space as real planes
// (Theory section, the linear system for X_p): occupied p gives the unit vector
// e_p; virtual p (a = p - o) gives [a_p, T]|Phi>: b(1h)_i = t_i^a and, in the
// doublet basis, b(2h1p)_ijb = t_ij^ab.
__global__ void rhs_rows_kernel(const int64_t* __restrict__ orb, const double* __restrict__ t1,
                                const double* __restrict__ t2, double* __restrict__ out, int64_t o, int64_t v,
                                int64_t o_pad, int64_t Dp) {
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
      if (t < o) {
        val = t1[t * v + a];
      } else if (t >= o_pad && t - o_pad < oov) {
        const int64_t idx = t - o_pad, ij = idx / v, b = idx % v;
        val = t2[(ij * v + a) * v + b];  // t2[i, j, a, b] at row (i, j, b)
      }
    }
    row[t] = val;
  }
}

// Left vectors c_q = <Phi|(1 + Lambda) abar_q^+ as real planes: occupied q from the
// rows built with the intermediates; virtual q (a = q - o): abar_q^+ = a_q^+ and
// c(1h)_i = l_i^a, c(2h1p)_klc = 2 l_kl^ac - l_kl^ca.
__global__ void left_rows_kernel(const int64_t* __restrict__ orb, const double* __restrict__ left_occ,
                                 const double* __restrict__ l1, const double* __restrict__ l2,
                                 double* __restrict__ out, int64_t o, int64_t v, int64_t o_pad, int64_t Dp) {
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
        val = 2.0 * l2[(kl * v + a) * v + cc] - l2[(kl * v + cc) * v + a];
      }
    }
    row[t] = val;
  }
}

void make_rhs_rows(gfcc_ctx* c, int64_t n, const int64_t* orb_dev, double* out, hipStream_t s) {
  if (n <= 0) return;
  if (c->sector != 0) {
    if (c->sector == 1)
      ea_rhs_rows(c, n, orb_dev, out, s);
    else
      uhf_rhs_rows(c, n, orb_dev, out, s);
    return;
  }
  hipLaunchKernelGGL(rhs_rows_kernel, dim3(blocks_for(c->Dp), unsigned(n)), dim3(256), 0, s, orb_dev,
                     c->t1c.as<double>(), c->t2, out, c->o, c->v, c->o_pad, c->Dp);
  GFCC_HIP(hipGetLastError());
}

void make_left_rows(gfcc_ctx* c, int64_t n, const int64_t* orb_dev, double* out, hipStream_t s) {
  if (n <= 0) return;
  if (c->sector != 0) {
    if (c->sector == 1)
      ea_left_rows(c, n, orb_dev, out, s);
    else
      uhf_left_rows(c, n, orb_dev, out, s);
    return;
  }
  hipLaunchKernelGGL(left_rows_kernel, dim3(blocks_for(c->Dp), unsigned(n)), dim3(256), 0, s, orb_dev,
                     c->left.as<double>(), c->l1c.as<double>(), c->l2 ? c->l2 : c->t2, out, c->o, c->v, c->o_pad,
                     c->Dp);
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

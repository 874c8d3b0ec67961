// Multi-shift GMRES: one Krylov basis per orbital serves every frequency.
//
// The Green's function comes from shifted linear systems (Introduction: they
// can be solved together over many frequencies; Theory section, the linear
// system for X_p).  The Krylov space of (omega - i eta + Hbar_N) and b_p does not
// depend on the shift, so the Arnoldi relation Hbar_N V_m = V_{m+1} Ht_m of ONE
// real basis (Hbar_N and b_p are real) serves every shift z = omega - i eta:
// (z + Hbar_N) V_m = V_{m+1} (Ht_m + z I~), and the GMRES iterate of shift z is
// X(z) = V_m y(z) with y(z) minimising |beta e_1 - (Ht_m + z I~) y|.  There is no
// preconditioner: the diagonal one depends on omega and would break the shared
// basis.  Nothing is restarted, so the basis grows to the largest iteration
// count any shift needs.
//
// Per orbital slot the library keeps V (orthonormal basis) and W = Hbar_N V (the
// sigma products before orthogonalisation), both FP64 planes.  Orthogonalisation
// is classical Gram-Schmidt twice, the second projection taken from the Gram
// matrix (V^T (w - V h1) = h1 - G h1, G = V^T V), so one step reads the basis
// twice.  The Hessenberg least-squares problems of all shifts are advanced on
// the host with complex Givens rotations, O(m) per shift and step.  When every
// shift of a slot has met its tolerance the true residual of each shift is
// formed in FP64 from the stored products, r(z) = b - V (z y) - W y (two GEMMs,
// no further sigma), and G_qp(omega) = (c_q^T V) y.
#include <algorithm>
#include <cmath>
#include <complex>
#include <map>
#include <vector>

#include "ctx.h"

namespace gfcc {

namespace {

using cd = std::complex<double>;

constexpr int VT = 256;          // threads per block
constexpr int VE = 8;            // elements per thread
constexpr int CH = VT * VE;      // elements per chunk
constexpr int KMAX = 512;        // largest Krylov dimension
constexpr int PSTR = 2 * (KMAX + 1);  // partial-dot stride per chunk

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
  return x;
}

struct MsDev {
  double* V;       // [B][K+1][Dp]
  double* W;       // [B][K][Dp]
  double* part;    // [na][nch][PSTR]  <V_j, w> at j, <V_j, V_m> at KMAX+1+j
  double* Gm;      // [B][K+1][K+1]    Gm[s][m][j] = <V_j, V_m>, j <= m
  double* h;       // [na][KMAX+1]
  double* npart;   // [na][nch]
  double* nrm;     // [na]
  const int* act;  // [na] slot of active entry
  const int* step; // [na] Krylov step m of active entry
  int K;
  int64_t Dp;
  int nch;
};

__device__ __forceinline__ double* vrow(const MsDev& d, int s, int j) {
  return d.V + (int64_t(s) * (d.K + 1) + j) * d.Dp;
}

// V[s][0] = b / |b|: e_p when brow < 0, else row brow of `brows`
__global__ void ms_init_kernel(MsDev d, const int* slots, const int* ps, const int* brow, const double* brows,
                               const double* bnorm, int n) {
  const int q = blockIdx.y;
  if (q >= n) return;
  const int s = slots[q];
  const int br = brow[q];
  const double* b = br < 0 ? nullptr : brows + int64_t(br) * d.Dp;
  const double f = br < 0 ? 1.0 : 1.0 / bnorm[br];
  double* v0 = vrow(d, s, 0);
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < d.Dp; t += int64_t(gridDim.x) * blockDim.x)
    v0[t] = b ? b[t] * f : (t == ps[q] ? 1.0 : 0.0);
}

// sigma input planes: win[i] = V[act[i]][step[i]]
__global__ void ms_gather_kernel(MsDev d, double* win) {
  const int i = blockIdx.y;
  const double* v = vrow(d, d.act[i], d.step[i]);
  double* u = win + int64_t(i) * d.Dp;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < d.Dp; t += int64_t(gridDim.x) * blockDim.x)
    u[t] = v[t];
}

// Pass 0: W[s][m] = w; chunk partials of <V_j, w> and <V_j, V_m> for j <= m.
__global__ __launch_bounds__(VT) void ms_dots_kernel(MsDev d, const double* wout) {
  const int i = blockIdx.y;
  const int s = d.act[i], m = d.step[i];
  const int64_t i0 = int64_t(blockIdx.x) * CH;
  const double* w = wout + int64_t(i) * d.Dp;
  double* wst = d.W + (int64_t(s) * d.K + m) * d.Dp;
  const double* vm = vrow(d, s, m);
  double x[VE], k[VE];
#pragma unroll
  for (int e = 0; e < VE; ++e) {
    const int64_t t = i0 + threadIdx.x + e * VT;
    x[e] = t < d.Dp ? w[t] : 0.0;
    k[e] = t < d.Dp ? vm[t] : 0.0;
    if (t < d.Dp) wst[t] = x[e];
  }
  __shared__ double lds[VT / 64][KMAX + 1][2];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int j = 0; j <= m; ++j) {
    const double* vj = vrow(d, s, j);
    double a = 0.0, g = 0.0;
#pragma unroll
    for (int e = 0; e < VE; ++e) {
      const int64_t t = i0 + threadIdx.x + e * VT;
      if (t < d.Dp) {
        const double u = vj[t];
        a += u * x[e];
        g += u * k[e];
      }
    }
    a = wave_sum(a);
    g = wave_sum(g);
    if (lane == 0) {
      lds[wv][j][0] = a;
      lds[wv][j][1] = g;
    }
  }
  __syncthreads();
  double* pp = d.part + (int64_t(i) * d.nch + blockIdx.x) * PSTR;
  for (int j = threadIdx.x; j <= m; j += VT) {
    double a = 0.0, g = 0.0;
    for (int u = 0; u < VT / 64; ++u) {
      a += lds[u][j][0];
      g += lds[u][j][1];
    }
    pp[j] = a;
    pp[KMAX + 1 + j] = g;
  }
}

// Per active entry: h1 and the new Gram column from the chunk partials, then
// h = 2 h1 - G h1 (G symmetric, Gm[s][i][j] = G(j, i) for j <= i).
__global__ __launch_bounds__(VT) void ms_reduce_kernel(MsDev d) {
  const int i = blockIdx.x;
  const int s = d.act[i], m = d.step[i];
  __shared__ double h1[KMAX + 1];
  double* Gcol = d.Gm + (int64_t(s) * (d.K + 1) + m) * (d.K + 1);
  for (int j = threadIdx.x; j <= m; j += VT) {
    double a = 0.0, g = 0.0;
    for (int c = 0; c < d.nch; ++c) {
      const double* pp = d.part + (int64_t(i) * d.nch + c) * PSTR;
      a += pp[j];
      g += pp[KMAX + 1 + j];
    }
    h1[j] = a;
    Gcol[j] = g;
  }
  __syncthreads();
  for (int j = threadIdx.x; j <= m; j += VT) {
    double gh = 0.0;
    for (int l = 0; l <= m; ++l) {
      const double gjl = j <= l ? d.Gm[(int64_t(s) * (d.K + 1) + l) * (d.K + 1) + j]
                                : d.Gm[(int64_t(s) * (d.K + 1) + j) * (d.K + 1) + l];
      gh += gjl * h1[l];
    }
    d.h[int64_t(i) * (KMAX + 1) + j] = 2.0 * h1[j] - gh;
  }
}

// Pass 2: V[s][m+1] = w - sum_j h_j V_j (unnormalised); chunk partials of its norm.
__global__ __launch_bounds__(VT) void ms_update_kernel(MsDev d, const double* wout) {
  const int i = blockIdx.y;
  const int s = d.act[i], m = d.step[i];
  const int64_t i0 = int64_t(blockIdx.x) * CH;
  const double* w = wout + int64_t(i) * d.Dp;
  const double* h = d.h + int64_t(i) * (KMAX + 1);
  double x[VE];
#pragma unroll
  for (int e = 0; e < VE; ++e) {
    const int64_t t = i0 + threadIdx.x + e * VT;
    x[e] = t < d.Dp ? w[t] : 0.0;
  }
  for (int j = 0; j <= m; ++j) {
    const double hj = h[j];
    const double* vj = vrow(d, s, j);
#pragma unroll
    for (int e = 0; e < VE; ++e) {
      const int64_t t = i0 + threadIdx.x + e * VT;
      if (t < d.Dp) x[e] -= hj * vj[t];
    }
  }
  double* out = vrow(d, s, m + 1);
  double acc = 0.0;
#pragma unroll
  for (int e = 0; e < VE; ++e) {
    const int64_t t = i0 + threadIdx.x + e * VT;
    if (t < d.Dp) out[t] = x[e];
    acc += x[e] * x[e];
  }
  __shared__ double red[VT / 64];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int u = 0; u < VT / 64; ++u) t += red[u];
    d.npart[int64_t(i) * d.nch + blockIdx.x] = t;
  }
}

__global__ void ms_norm_kernel(MsDev d) {
  const int i = blockIdx.x;
  __shared__ double red[64];
  double acc = 0.0;
  for (int c = threadIdx.x; c < d.nch; c += 64) acc += d.npart[int64_t(i) * d.nch + c];
  red[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int u = 0; u < 64; ++u) t += red[u];
    d.nrm[i] = sqrt(t);
  }
}

// V[s][m+1] /= |V[s][m+1]| (left as is when the norm vanishes: breakdown)
__global__ void ms_scale_kernel(MsDev d) {
  const int i = blockIdx.y;
  const double n = d.nrm[i];
  const double f = n > 0.0 ? 1.0 / n : 1.0;
  double* v = vrow(d, d.act[i], d.step[i] + 1);
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < d.Dp; t += int64_t(gridDim.x) * blockDim.x)
    v[t] *= f;
}

// Residual planes R[2k], R[2k+1] (re, im of shift k = blockIdx.y) plus b: partial
// squared norms of RB slices of the plane, out[k][blockIdx.x].
constexpr int RB = 64;
__global__ void ms_resid_kernel(const double* R, int64_t Dp, const double* b, int p, double* out) {
  const int k = blockIdx.y;
  const double* rr = R + (int64_t(2) * k) * Dp;
  const double* ri = rr + Dp;
  const int64_t len = (Dp + RB - 1) / RB;
  const int64_t t0 = int64_t(blockIdx.x) * len, t1 = std::min<int64_t>(Dp, t0 + len);
  double acc = 0.0;
  for (int64_t t = t0 + threadIdx.x; t < t1; t += VT) {
    const double bt = b ? b[t] : (t == p ? 1.0 : 0.0);
    const double a = rr[t] + bt, c = ri[t];
    acc += a * a + c * c;
  }
  __shared__ double red[VT / 64];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int u = 0; u < VT / 64; ++u) t += red[u];
    out[int64_t(k) * RB + blockIdx.x] = t;
  }
}

// |row r| of rows [n][Dp]
__global__ void ms_rownorm_kernel(const double* rows, int64_t Dp, double* out) {
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
    double t = 0.0;
    for (int u = 0; u < VT / 64; ++u) t += red[u];
    out[r] = sqrt(t);
  }
}

unsigned grid_for(int64_t n) { return unsigned(std::min<int64_t>((n + 255) / 256, 1024)); }

template <typename T>
void upload(DBuf& b, const std::vector<T>& v, hipStream_t s) {
  b.ensure(std::max<size_t>(v.size(), 1) * sizeof(T), s);
  if (!v.empty()) GFCC_HIP(hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

// Givens state of one shift: rotations of the columns processed so far and the
// rotated right-hand side g.
struct Shift {
  cd z;
  int ncol = 0;          // Hessenberg columns applied
  int m_used = 0;        // basis size of the accepted iterate (0: not yet)
  double target = 0.0;   // residual-estimate target (absolute)
  double est = 0.0;      // |g_{ncol}|
  std::vector<cd> cs, sn, g;
};

// Upper Hessenberg column j (rows 0..j+1) of the real basis, shifted by z.
void apply_column(Shift& sh, const std::vector<double>& H, int ldH, int j) {
  thread_local std::vector<cd> col;
  col.resize(size_t(j) + 2);
  for (int i = 0; i <= j + 1; ++i) col[size_t(i)] = cd(H[size_t(j) * ldH + i], 0.0);
  col[size_t(j)] += sh.z;
  for (int i = 0; i < j; ++i) {
    const cd a = sh.cs[size_t(i)] * col[size_t(i)] + sh.sn[size_t(i)] * col[size_t(i) + 1];
    col[size_t(i) + 1] = -std::conj(sh.sn[size_t(i)]) * col[size_t(i)] + std::conj(sh.cs[size_t(i)]) * col[size_t(i) + 1];
    col[size_t(i)] = a;
  }
  const double r = std::hypot(std::abs(col[size_t(j)]), std::abs(col[size_t(j) + 1]));
  cd c(1.0, 0.0), sn(0.0, 0.0);
  if (r > 0.0) {
    c = std::conj(col[size_t(j)]) / r;
    sn = std::conj(col[size_t(j) + 1]) / r;
  }
  sh.cs.push_back(c);
  sh.sn.push_back(sn);
  const cd gj = sh.g[size_t(j)];
  sh.g.push_back(-std::conj(sn) * gj);
  sh.g[size_t(j)] = c * gj;
  sh.ncol = j + 1;
  sh.est = std::abs(sh.g[size_t(j) + 1]);
}

// y minimising |beta e1 - (Ht_m + z I~) y| for the first m columns (a fresh QR:
// the running rotations are not kept as a triangle).
std::vector<cd> solve_small(const std::vector<double>& H, int ldH, int m, cd z, double beta) {
  std::vector<cd> R(size_t(m) * m), g(size_t(m) + 1, cd(0.0, 0.0));
  std::vector<cd> cs(static_cast<size_t>(m)), sn(static_cast<size_t>(m));
  g[0] = beta;
  for (int j = 0; j < m; ++j) {
    std::vector<cd> col(size_t(j) + 2);
    for (int i = 0; i <= j + 1; ++i) col[size_t(i)] = cd(H[size_t(j) * ldH + i], 0.0);
    col[size_t(j)] += z;
    for (int i = 0; i < j; ++i) {
      const cd a = cs[size_t(i)] * col[size_t(i)] + sn[size_t(i)] * col[size_t(i) + 1];
      col[size_t(i) + 1] = -std::conj(sn[size_t(i)]) * col[size_t(i)] + std::conj(cs[size_t(i)]) * col[size_t(i) + 1];
      col[size_t(i)] = a;
    }
    const double r = std::hypot(std::abs(col[size_t(j)]), std::abs(col[size_t(j) + 1]));
    cd c(1.0, 0.0), s(0.0, 0.0);
    if (r > 0.0) {
      c = std::conj(col[size_t(j)]) / r;
      s = std::conj(col[size_t(j) + 1]) / r;
    }
    cs[size_t(j)] = c;
    sn[size_t(j)] = s;
    col[size_t(j)] = c * col[size_t(j)] + s * col[size_t(j) + 1];
    const cd gj = g[size_t(j)];
    g[size_t(j) + 1] = -std::conj(s) * gj;
    g[size_t(j)] = c * gj;
    for (int i = 0; i <= j; ++i) R[size_t(j) * m + i] = col[size_t(i)];
  }
  std::vector<cd> y(static_cast<size_t>(m));
  for (int i = m - 1; i >= 0; --i) {
    cd acc = g[size_t(i)];
    for (int j = i + 1; j < m; ++j) acc -= R[size_t(j) * m + i] * y[size_t(j)];
    const cd d = R[size_t(i) * m + i];
    y[size_t(i)] = std::abs(d) > 0.0 ? acc / d : cd(0.0, 0.0);
  }
  return y;
}

struct Slot {
  int64_t pi = -1;  // index into the caller's p list
  int m = 0;        // basis vectors built (V_0..V_m valid, W_0..W_{m-1})
  double bn = 1.0;
  int brow = -1;
  bool breakdown = false;
  std::vector<double> H;  // column j at H[j * (K + 2)], rows 0..j+1
  std::vector<Shift> sh;
};

}  // namespace

void solve_shifts(gfcc_ctx* c, int64_t np, const int64_t* p, int64_t nw, const double* omega, double eta,
                  int64_t nq, const int64_t* q, const gfcc_shift_opts* o, double* G, double* Xout,
                  gfcc_rhs_info* info, hipStream_t s, bool* all_converged) {
  const int64_t Dp = c->Dp, D = c->D;
  const int K = o->max_dim > 0 ? int(std::min<int64_t>(o->max_dim, KMAX)) : 160;
  const int ldH = K + 2;
  const int nch = int((Dp + CH - 1) / CH);
  const double tol = o->tol;
  const int64_t nql = q ? nq : 1;
  const int64_t KC = 64;  // shifts per verification / X chunk

  int B = o->batch > 0 ? int(o->batch) : 0;
  if (B == 0) {
    size_t freeb = 0, totalb = 0;
    GFCC_HIP(hipMemGetInfo(&freeb, &totalb));
    const double per_slot = double(2 * K + 1) * Dp * 8.0 + double(K + 1) * (K + 1) * 8.0;
    B = int(std::max<int64_t>(1, std::min<int64_t>(int64_t(0.4 * double(freeb) / per_slot), 256)));
  }
  B = int(std::min<int64_t>(B, np));

  // right-hand sides of virtual orbitals (one plane per distinct orbital) and their norms
  std::map<int64_t, int> brow_of;
  std::vector<int64_t> borb;
  for (int64_t r = 0; r < np; ++r)
    if (c->materialised(p[r]) && !brow_of.count(p[r])) {
      brow_of[p[r]] = int(borb.size());
      borb.push_back(p[r]);
    }
  DBuf d_borb, bB, bBn;
  std::vector<double> bnorm_h(borb.size());
  if (!borb.empty()) {
    const int64_t nb = int64_t(borb.size());
    upload(d_borb, borb, s);
    bB.ensure(size_t(nb * Dp) * 8, s);
    bBn.ensure(size_t(nb) * 8, s);
    make_rhs_rows(c, nb, d_borb.as<int64_t>(), bB.as<double>(), s);
    hipLaunchKernelGGL(ms_rownorm_kernel, dim3(unsigned(nb)), dim3(VT), 0, s, bB.as<double>(), Dp, bBn.as<double>());
    GFCC_HIP(hipGetLastError());
    GFCC_HIP(hipMemcpyAsync(bnorm_h.data(), bBn.p, size_t(nb) * 8, hipMemcpyDeviceToHost, s));
  }
  // left vectors: one plane per distinct q (or per distinct p when q == NULL)
  std::map<int64_t, int64_t> lrow_of;
  std::vector<int64_t> lorb;
  for (int64_t k = 0; k < (q ? nq : np); ++k) {
    const int64_t orb = q ? q[k] : p[k];
    if (!lrow_of.count(orb)) {
      lrow_of[orb] = int64_t(lorb.size());
      lorb.push_back(orb);
    }
  }
  DBuf d_lorb, bL;
  upload(d_lorb, lorb, s);
  bL.ensure(lorb.size() * size_t(Dp) * 8, s);
  make_left_rows(c, int64_t(lorb.size()), d_lorb.as<int64_t>(), bL.as<double>(), s);
  std::vector<int64_t> qrow(static_cast<size_t>(nql));
  if (q)
    for (int64_t k = 0; k < nq; ++k) qrow[size_t(k)] = lrow_of.at(q[k]);

  // device state
  DBuf bV, bW, bpart, bGm, bh, bnpart, bnrm, d_act, d_step, d_list, d_plist, d_brow;
  bV.ensure(size_t(B) * (K + 1) * Dp * 8, s);
  bW.ensure(size_t(B) * K * Dp * 8, s);
  bpart.ensure(size_t(B) * nch * PSTR * 8, s);
  bGm.ensure(size_t(B) * (K + 1) * (K + 1) * 8, s);
  bh.ensure(size_t(B) * (KMAX + 1) * 8, s);
  bnpart.ensure(size_t(B) * nch * 8, s);
  bnrm.ensure(size_t(B) * 8, s);
  c->ws_in.ensure(size_t(B) * Dp * 8, s);
  c->ws_out.ensure(size_t(B) * Dp * 8, s);
  MsDev d;
  d.V = bV.as<double>();
  d.W = bW.as<double>();
  d.part = bpart.as<double>();
  d.Gm = bGm.as<double>();
  d.h = bh.as<double>();
  d.npart = bnpart.as<double>();
  d.nrm = bnrm.as<double>();
  d.K = K;
  d.Dp = Dp;
  d.nch = nch;
  Scratch scr;
  DBuf bcoef, bR, bCV, brn;
  GFCC_HIP(hipStreamSynchronize(s));

  for (int64_t r = 0; r < np * nw; ++r) info[r] = gfcc_rhs_info{1, 0, 0, 0, 0.0};
  std::vector<Slot> slots(static_cast<size_t>(B));
  std::vector<int> free_slots, active;
  for (int i = B - 1; i >= 0; --i) free_slots.push_back(i);
  std::vector<std::pair<int64_t, int64_t>> failed;  // (orbital index, shift) left for the fallback
  int64_t next = 0;

  auto refill = [&]() {
    std::vector<int> sl, pl, bl;
    while (!free_slots.empty() && next < np) {
      const int br = c->materialised(p[next]) ? brow_of.at(p[next]) : -1;
      const double bn = br < 0 ? 1.0 : bnorm_h[size_t(br)];
      if (!(bn > 0.0)) {  // b_p = 0: X = 0 and G = 0 at every shift
        GFCC_HIP(hipMemsetAsync(G + next * nw * nql * 2, 0, size_t(nw * nql) * 16, s));
        if (Xout) GFCC_HIP(hipMemsetAsync(Xout + next * nw * D * 2, 0, size_t(nw * D) * 16, s));
        for (int64_t k = 0; k < nw; ++k) info[next * nw + k] = gfcc_rhs_info{0, 0, 0, 0, 0.0};
        ++next;
        continue;
      }
      const int si = free_slots.back();
      free_slots.pop_back();
      Slot& S = slots[size_t(si)];
      S = Slot{};
      S.pi = next;
      S.bn = bn;
      S.brow = br;
      S.H.assign(size_t(K) * ldH, 0.0);
      S.sh.resize(size_t(nw));
      for (int64_t k = 0; k < nw; ++k) {
        Shift& h = S.sh[size_t(k)];
        h.z = cd(omega[k], -eta);
        h.g.assign(1, cd(bn, 0.0));
        h.target = 0.5 * tol * bn;
        h.est = bn;
      }
      sl.push_back(si);
      pl.push_back(int(p[next]));
      bl.push_back(br);
      active.push_back(si);
      ++next;
    }
    if (sl.empty()) return;
    upload(d_list, sl, s);
    upload(d_plist, pl, s);
    upload(d_brow, bl, s);
    hipLaunchKernelGGL(ms_init_kernel, dim3(grid_for(Dp), unsigned(sl.size())), dim3(256), 0, s, d,
                       d_list.as<int>(), d_plist.as<int>(), d_brow.as<int>(), bB.as<double>(), bBn.as<double>(),
                       int(sl.size()));
    GFCC_HIP(hipGetLastError());
    GFCC_HIP(hipStreamSynchronize(s));  // host vectors above go out of scope
  };

  // GEMM R[2kc][Dp] = Cf[2kc][m] . rows[m][Dp] (+ beta R)
  auto comb = [&](const double* coef, int64_t ldc, int64_t rows2, int m, const double* rows, double beta,
                  double* R) {
    GemmArgs g;
    g.A = coef;
    g.am = lin(ldc);
    g.B = rows;
    g.bm = lin(Dp);
    g.b_ncontig = 1;
    g.M = rows2;
    g.N = Dp;
    g.K = m;
    g.C = R;
    g.cm = lin(Dp);
    g.cn = lin(1);
    g.alpha = 1.0;
    g.beta = beta;
    gemm(Prec::F64, g, gemm_default_cfg(rows2, Dp, m), s);
  };

  // Verify and finish a slot whose shifts all met their estimate (or that hit
  // K / broke down).  Returns false when some shift failed the true-residual
  // check and the basis can still grow.
  auto finish = [&](int si) -> bool {
    Slot& S = slots[size_t(si)];
    const int m = S.m;
    const double* Vs = d.V + int64_t(si) * (K + 1) * Dp;
    const double* Ws = d.W + int64_t(si) * K * Dp;
    const double* bptr = S.brow < 0 ? nullptr : bB.as<double>() + int64_t(S.brow) * Dp;
    std::vector<std::vector<cd>> Y(static_cast<size_t>(nw));
    std::vector<int> mu(static_cast<size_t>(nw));
    const int64_t ldc = (m + 7) / 8 * 8;
    std::vector<double> rel(static_cast<size_t>(nw));
    for (;;) {
      for (int64_t k = 0; k < nw; ++k) {
        const Shift& h = S.sh[size_t(k)];
        mu[size_t(k)] = h.m_used > 0 ? h.m_used : m;
        Y[size_t(k)] = solve_small(S.H, ldH, mu[size_t(k)], h.z, S.bn);
        Y[size_t(k)].resize(size_t(m), cd(0.0, 0.0));
      }
      if (o->verify) {
        bcoef.ensure(size_t(4 * KC * ldc) * 8, s);
        bR.ensure(size_t(2 * KC * Dp) * 8, s);
        brn.ensure(size_t(KC) * RB * 8, s);
        for (int64_t k0 = 0; k0 < nw; k0 += KC) {
          const int64_t kc = std::min(KC, nw - k0);
          std::vector<double> cf(size_t(4 * kc * ldc), 0.0);  // [Cv | Cw] row blocks
          double* cv = cf.data();
          double* cw = cf.data() + 2 * kc * ldc;
          for (int64_t k = 0; k < kc; ++k) {
            const cd z = S.sh[size_t(k0 + k)].z;
            for (int j = 0; j < m; ++j) {
              const cd y = Y[size_t(k0 + k)][size_t(j)];
              const cd zy = z * y;
              cv[(2 * k) * ldc + j] = -zy.real();
              cv[(2 * k + 1) * ldc + j] = -zy.imag();
              cw[(2 * k) * ldc + j] = -y.real();
              cw[(2 * k + 1) * ldc + j] = -y.imag();
            }
          }
          GFCC_HIP(hipMemcpyAsync(bcoef.p, cf.data(), cf.size() * 8, hipMemcpyHostToDevice, s));
          comb(bcoef.as<double>(), ldc, 2 * kc, m, Vs, 0.0, bR.as<double>());
          comb(bcoef.as<double>() + 2 * kc * ldc, ldc, 2 * kc, m, Ws, 1.0, bR.as<double>());
          hipLaunchKernelGGL(ms_resid_kernel, dim3(RB, unsigned(kc)), dim3(VT), 0, s, bR.as<double>(), Dp, bptr,
                             int(p[S.pi]), brn.as<double>());
          GFCC_HIP(hipGetLastError());
          std::vector<double> part(size_t(kc) * RB);
          GFCC_HIP(hipMemcpyAsync(part.data(), brn.p, part.size() * 8, hipMemcpyDeviceToHost, s));
          GFCC_HIP(hipStreamSynchronize(s));  // cf goes out of scope
          for (int64_t k = 0; k < kc; ++k) {
            double t = 0.0;
            for (int u = 0; u < RB; ++u) t += part[size_t(k * RB + u)];
            rel[size_t(k0 + k)] = std::sqrt(t);
          }
        }
        for (auto& r : rel) r /= S.bn;
      } else {
        for (int64_t k = 0; k < nw; ++k) {
          const Shift& h = S.sh[size_t(k)];
          rel[size_t(k)] = (h.m_used > 0 ? h.est : std::abs(h.g.back())) / S.bn;
        }
      }
      // A shift whose true residual misses the tolerance although its estimate
      // met it takes more columns: those already built, then new ones.
      bool changed = false, grow = false;
      if (m < K && !S.breakdown) {
        for (int64_t k = 0; k < nw; ++k) {
          Shift& h = S.sh[size_t(k)];
          if (rel[size_t(k)] <= tol || !std::isfinite(rel[size_t(k)]) || h.m_used == 0) continue;
          const int old = h.m_used;
          h.m_used = 0;
          h.target *= 0.1;
          for (int j = h.ncol; j < m; ++j) apply_column(h, S.H, ldH, j);
          if (h.ncol > old && h.est <= h.target) h.m_used = h.ncol;
          changed = true;
          grow = grow || h.m_used == 0;
        }
      }
      if (grow) return false;
      if (!changed) break;
    }

    // G_qp(omega_k) = sum_j (c_q . V_j) y_k[j]
    const int64_t nl = q ? int64_t(lorb.size()) : 1;
    bCV.ensure(size_t(nl * ldc) * 8, s);
    {
      GemmArgs g;
      g.A = q ? bL.as<double>() : bL.as<double>() + lrow_of.at(p[S.pi]) * Dp;
      g.am = lin(Dp);
      g.B = Vs;
      g.bm = lin(Dp);
      g.M = nl;
      g.N = m;
      g.K = Dp;
      g.C = bCV.as<double>();
      g.cm = lin(ldc);
      g.cn = lin(1);
      gemm_auto(Prec::F64, g, scr, 0, s);
    }
    std::vector<double> CV(size_t(nl * ldc));
    GFCC_HIP(hipMemcpyAsync(CV.data(), bCV.p, CV.size() * 8, hipMemcpyDeviceToHost, s));
    GFCC_HIP(hipStreamSynchronize(s));
    std::vector<double> Gh(size_t(nw * nql * 2));
    for (int64_t k = 0; k < nw; ++k)
      for (int64_t t = 0; t < nql; ++t) {
        const double* cv = CV.data() + (q ? qrow[size_t(t)] : 0) * ldc;
        cd acc(0.0, 0.0);
        for (int j = 0; j < m; ++j) acc += cv[j] * Y[size_t(k)][size_t(j)];
        Gh[size_t((k * nql + t) * 2)] = acc.real();
        Gh[size_t((k * nql + t) * 2 + 1)] = acc.imag();
      }
    GFCC_HIP(hipMemcpyAsync(G + S.pi * nw * nql * 2, Gh.data(), Gh.size() * 8, hipMemcpyHostToDevice, s));
    if (Xout) {  // X(omega_k) = V y_k
      bcoef.ensure(size_t(4 * KC * ldc) * 8, s);
      bR.ensure(size_t(2 * KC * Dp) * 8, s);
      for (int64_t k0 = 0; k0 < nw; k0 += KC) {
        const int64_t kc = std::min(KC, nw - k0);
        std::vector<double> cf(size_t(2 * kc * ldc), 0.0);
        for (int64_t k = 0; k < kc; ++k)
          for (int j = 0; j < m; ++j) {
            cf[size_t((2 * k) * ldc + j)] = Y[size_t(k0 + k)][size_t(j)].real();
            cf[size_t((2 * k + 1) * ldc + j)] = Y[size_t(k0 + k)][size_t(j)].imag();
          }
        GFCC_HIP(hipMemcpyAsync(bcoef.p, cf.data(), cf.size() * 8, hipMemcpyHostToDevice, s));
        comb(bcoef.as<double>(), ldc, 2 * kc, m, Vs, 0.0, bR.as<double>());
        from_planes(c, kc, bR.as<double>(), Xout + (S.pi * nw + k0) * D * 2, s);
        GFCC_HIP(hipStreamSynchronize(s));
      }
    }
    for (int64_t k = 0; k < nw; ++k) {
      const double r = rel[size_t(k)];
      const int st = !std::isfinite(r) ? 3 : (r <= tol ? 0 : 1);
      info[S.pi * nw + k] = gfcc_rhs_info{st, mu[size_t(k)], 0, 0, r};
      if (st != 0) failed.push_back({S.pi, k});
    }
    GFCC_HIP(hipStreamSynchronize(s));  // Gh goes out of scope
    return true;
  };

  if (o->tune_cache && c->sector == 0) {  // FP64 sigma tiles for a full orbital window
    tune_load(c, o->tune_cache);
    tune_ring(c, Prec::F64, int64_t(B), s);
    tune_save(c, o->tune_cache);
  }
  refill();
  std::vector<double> hh(size_t(B) * (KMAX + 1)), hn(static_cast<size_t>(B));
  while (!active.empty()) {
    const int na = int(active.size());
    std::vector<int> st(static_cast<size_t>(na));
    for (int i = 0; i < na; ++i) st[size_t(i)] = slots[size_t(active[size_t(i)])].m;
    upload(d_act, active, s);
    upload(d_step, st, s);
    d.act = d_act.as<int>();
    d.step = d_step.as<int>();
    hipLaunchKernelGGL(ms_gather_kernel, dim3(grid_for(Dp), unsigned(na)), dim3(256), 0, s, d, c->ws_in.as<double>());
    GFCC_HIP(hipGetLastError());
    sigma_planes(c, na, c->ws_in.as<double>(), c->ws_out.as<double>(), GFCC_FP64, s);
    prof_begin(c, "arnoldi_shifts", s);
    hipLaunchKernelGGL(ms_dots_kernel, dim3(unsigned(nch), unsigned(na)), dim3(VT), 0, s, d, c->ws_out.as<double>());
    hipLaunchKernelGGL(ms_reduce_kernel, dim3(unsigned(na)), dim3(VT), 0, s, d);
    hipLaunchKernelGGL(ms_update_kernel, dim3(unsigned(nch), unsigned(na)), dim3(VT), 0, s, d, c->ws_out.as<double>());
    hipLaunchKernelGGL(ms_norm_kernel, dim3(unsigned(na)), dim3(64), 0, s, d);
    hipLaunchKernelGGL(ms_scale_kernel, dim3(grid_for(Dp), unsigned(na)), dim3(256), 0, s, d);
    GFCC_HIP(hipGetLastError());
    prof_end(c, "arnoldi_shifts", s, 0.0, 0.0);
    GFCC_HIP(hipMemcpyAsync(hh.data(), bh.p, size_t(na) * (KMAX + 1) * 8, hipMemcpyDeviceToHost, s));
    GFCC_HIP(hipMemcpyAsync(hn.data(), bnrm.p, size_t(na) * 8, hipMemcpyDeviceToHost, s));
    GFCC_HIP(hipStreamSynchronize(s));

    std::vector<int> still, done;
    for (int i = 0; i < na; ++i) {
      const int si = active[size_t(i)];
      Slot& S = slots[size_t(si)];
      const int j = S.m;
      double hmax = 0.0;
      for (int l = 0; l <= j; ++l) {
        S.H[size_t(j) * ldH + l] = hh[size_t(i) * (KMAX + 1) + l];
        hmax = std::max(hmax, std::fabs(hh[size_t(i) * (KMAX + 1) + l]));
      }
      S.H[size_t(j) * ldH + j + 1] = hn[size_t(i)];
      S.m = j + 1;
      if (!(hn[size_t(i)] > 1e-14 * std::max(hmax, 1e-300))) S.breakdown = true;
      bool all = true;
      for (auto& h : S.sh) {
        if (h.m_used > 0) continue;
        apply_column(h, S.H, ldH, j);
        if (h.est <= h.target || S.breakdown) h.m_used = h.ncol;
        all = all && h.m_used > 0;
      }
      if (all || S.m >= K || S.breakdown)
        done.push_back(si);
      else
        still.push_back(si);
    }
    for (int si : done) {
      if (finish(si)) {
        slots[size_t(si)].pi = -1;
        free_slots.push_back(si);
      } else {
        still.push_back(si);
      }
    }
    active.swap(still);
    refill();
  }

  // shifts that did not converge within K basis vectors: restarted preconditioned solves
  if (!failed.empty() && o->use_fallback) {
    const int64_t nf = int64_t(failed.size());
    std::vector<int64_t> Pf(static_cast<size_t>(nf));
    std::vector<double> Wf(static_cast<size_t>(nf));
    for (int64_t r = 0; r < nf; ++r) {
      Pf[size_t(r)] = p[failed[size_t(r)].first];
      Wf[size_t(r)] = omega[failed[size_t(r)].second];
    }
    DBuf Gf, Xf;
    Gf.ensure(size_t(nf * nql) * 16, s);
    if (Xout) Xf.ensure(size_t(nf * D) * 16, s);
    std::vector<gfcc_rhs_info> inf(static_cast<size_t>(nf));
    bool conv = true;
    gfcc_solve_opts fo = o->fallback;
    fo.checkpoint = nullptr;
    solve_batch(c, nf, Pf.data(), Wf.data(), eta, nql, q, &fo, Gf.as<double>(),
                Xout ? Xf.as<double>() : nullptr, inf.data(), s, &conv, nullptr);
    for (int64_t r = 0; r < nf; ++r) {
      const int64_t row = failed[size_t(r)].first * nw + failed[size_t(r)].second;
      GFCC_HIP(hipMemcpyAsync(G + row * nql * 2, Gf.as<double>() + r * nql * 2, size_t(nql) * 16,
                              hipMemcpyDeviceToDevice, s));
      if (Xout)
        GFCC_HIP(hipMemcpyAsync(Xout + row * D * 2, Xf.as<double>() + r * D * 2, size_t(D) * 16,
                                hipMemcpyDeviceToDevice, s));
      gfcc_rhs_info& x = info[row];
      const int m0 = x.iters;
      x = inf[size_t(r)];
      x.iters += m0;
      x.restarts += 1;
    }
    GFCC_HIP(hipStreamSynchronize(s));
  }
  bool ok = true;
  for (int64_t r = 0; r < np * nw; ++r) ok = ok && (info[r].status == 0 || info[r].status == 4);
  *all_converged = ok;
  GFCC_HIP(hipStreamSynchronize(s));
}

}  // namespace gfcc

// The gfcc context: per-system intermediates in HBM plus reusable workspaces.
#pragma once
#include <map>
#include <string>

#include "gfcc_internal.h"
#include "mlp.h"
#include "mor.h"

struct gfcc_prof_entry {
  int64_t count = 0;
  double ms = 0.0, flops = 0.0, bytes = 0.0;
};

struct gfcc_ctx {
  // dimensions
  int64_t o = 0, v = 0, Q = 0, n = 0, D = 0;
  int64_t ov = 0, oo = 0, oov = 0;
  int64_t o_pad = 0;  // start of the 2h1p block inside a plane
  int64_t Dp = 0;     // plane length (re or im part of one vector)
  int64_t kp = 0;     // padded length of an (m,e) index range: round8(o v)
  int64_t k2 = 0;     // row length of the ring matrix: 2 kp
  int64_t op2 = 0;    // padded row length of [o^2][o^2] / [v][o^2] operands
  int64_t vp = 0;     // padded row length for K = v operands
  int64_t Qp = 0;     // padded Cholesky rank (rows of Q-innermost operands)

  // Sector of the expansion: 0 = ionisation (1h + 2h1p), 1 = electron attachment (1p + 2p1h),
  // 2 = ionisation of an open-shell reference over spin orbitals (1h + 2h1p, both pair orders).
  // A plane holds the first block at [0, n1) and the second at [p1, p1 + n2); D = n1 + n2.
  int sector = 0;
  int64_t n1 = 0, p1 = 0, n2 = 0;
  // right-hand side (and left vector) of orbital `orb` is a materialised row rather than the
  // implicit unit vector of an occupied orbital of the IP sector
  bool materialised(int64_t orb) const { return sector != 0 || orb >= o; }

  // borrowed inputs (caller memory, valid until gfcc_destroy): t2, and l2 when
  // Lambda is not T^dagger (else nullptr)
  const double* t2 = nullptr;
  const double* l2 = nullptr;

  // FP64 blocks (natural layouts, see gfcc_export)
  gfcc::DBuf Foo, Fvv, Fov, Wooov;
  // ring matrix WW[(j,a)][0:kp) = Wovvo[m,a,e,j], WW[(j,a)][kp:2kp) = Wovov[m,a,j,e] (+ folds),
  // columns (m,e); sigma's first ring product reads whole rows against [2R - RT | -R]
  gfcc::DBuf WW;
  gfcc::DBuf W4T;     // [(i,j)][op2]     W4T[(i,j)][(m,n)] = Woooo[m,n,i,j]
  gfcc::DBuf WovooT;  // [(i,j,a)][o_pad] WovooT[(i,j,a)][m] = Wovoo[m,a,i,j]
  gfcc::DBuf LovC;    // [Q][kp]          L[Q][m][o+e] at column (m,e) (three-body, first half)
  gfcc::DBuf LovT;    // [v][o][Qp]       L[Q][m][o+e] at [e][m][Q]   (three-body, second half)
  gfcc::DBuf d1b;     // [(i,j,a)]        Fvv[a,a] - Foo[i,i] - Foo[j,j]
  gfcc::DBuf Uop;     // [o][Dp]          1h rows of Hbar_N over a plane
  gfcc::DBuf diag;    // [Dp]             exact diagonal (1.0 in padding)
  gfcc::DBuf left;    // [o][Dp]          c_q rows
  gfcc::DBuf t1c;     // [o][v]           amplitudes for virtual-orbital right-hand sides
  gfcc::DBuf l1c;     // [o][v]

  // electron-attachment blocks (sector 1), FP64
  struct EA {
    int64_t lv = 0;     // row stride of the ladder matrix: round8(v^2)
    int64_t n2p = 0;    // row stride of zop: round8(o v^2)
    gfcc::DBuf ladder;  // [(a,b)][lv]    Wvvvv[a,b,c,d] at column (c,d)
    gfcc::DBuf vvvoT;   // [(j,a,b)][vp]  Wvvvo[a,b,c,j] at column c
    gfcc::DBuf ring;    // [(j,b)][2kp]   [2 Wovvo[l,b,d,j] - Wovov[l,b,j,d] (+ one-body) | -Wovvo[l,b,c,j]]
    gfcc::DBuf ring2;   // [(j,a)][kp]    -Wovov[l,a,j,c] (+ one-body)
    gfcc::DBuf zop;     // [k][n2p]       2 (kc|ld) - (kd|lc) at column (l,c,d)
    gfcc::DBuf Sl;      // [a][b]         sum_ijc t2[i,j,a,c] (2 l2[i,j,b,c] - l2[i,j,c,b])
    gfcc::DBuf ws_R, ws_z;  // sigma operand copies
    // FP16 copies for the FP16-IR form (per-tensor power-of-two scales, stored = value * s)
    struct Half {
      bool built = false;
      gfcc::DBuf ladder, vvvoT, Uop, ring, ring2, zop, t2;
      double sL = 1, sV = 1, sU = 1, sR = 1, sR2 = 1, sZ = 1, sT = 1;
    } h;
    gfcc::DBuf ws_xh, ws_Rh, ws_zh;  // FP16 operand copies of a sigma call
  } ea;

  // open-shell (spin-unrestricted) IP blocks (sector 2), FP64, over spin orbitals
  struct UHF {
    gfcc::DBuf t1, t2, l1, l2;              // spin-orbital amplitudes [o][v], [o][o][v][v]
    gfcc::DBuf oovv, Woooo, Wooov, Wovvo, Wovoo;
    gfcc::DBuf S;                           // [i][q] left-vector helper
    gfcc::DBuf ws_z;                        // sigma three-body intermediate
  } uhf;

  // reduced-precision copies of the two-body operands with power-of-two scales: [0] FP32, [1] BF16, [2] FP16
  struct LowPrec {
    bool built = false;
    gfcc::DBuf WW, W4T, WovooT, t2, LovC;
    double sWW = 1, sW4T = 1, sWovooT = 1, st2 = 1, sLovC = 1;  // stored = value * s
  } lp[3];

  // workspaces
  gfcc::Scratch scr;
  gfcc::DBuf ws_A1, ws_RT, ws_Ra, ws_r1, ws_U, ws_z, ws_zl;  // sigma operand copies
  gfcc::DBuf ws_in, ws_out;                 // planes for gfcc_sigma / gfcc_greens
  // FP16 sigma: device scales of the vector operands ([0] s, [1] 1/s, [2] s_z, [3] 1/(s s_z)) and
  // the per-block maxima they are reduced from
  gfcc::DBuf ws_vsc, ws_vpart;

  // kernel timing
  bool prof_on = false;
  std::map<std::string, gfcc_prof_entry> prof;
  std::map<std::string, std::vector<std::pair<hipEvent_t, hipEvent_t>>> prof_events;
  struct PendingMeta {
    double flops, bytes;
  };
  std::map<std::string, std::vector<PendingMeta>> prof_meta;

  // autotuned tile choice for the ring GEMMs, keyed "prec:M:N:K"
  std::map<std::string, int> tuned;
  std::map<std::string, float> tuned_ms;

  // learned preconditioner (created by training or by setting weights)
  std::unique_ptr<gfcc::Mlp> mlp;

  // model-order reduction basis and projected operator
  std::unique_ptr<gfcc::Mor> mor;

  // device of the context and the address there of the library's fixed scratch
  // array (the allocation-free entry points)
  int device = -1;
  void* fixed_scratch = nullptr;
};

namespace gfcc {
// Training data recorded by a solve: at every restart the true residual r_k and
// the iterate x_k of a right-hand side; X* when it converges.
struct PairRec {
  double* R = nullptr;      // [cap][2][Dp]
  double* X = nullptr;      // [cap][2][Dp]
  double* xstar = nullptr;  // [nrhs][2][Dp]
  int64_t cap = 0, n = 0;
  std::vector<int> rhs;
  std::vector<double> omega, nrm;
  // per right-hand side: |r| / sqrt(D) of the final iterate of a solve that stopped at max_iter
  // (its iterate is then kept in xstar too); 0 otherwise
  std::vector<double> final_nrm;
};
void solve_batch(gfcc_ctx* c, int64_t nrhs, const int64_t* p, const double* omega, double eta, int64_t nq,
                 const int64_t* q, const gfcc_solve_opts* opts, double* G, double* X, gfcc_rhs_info* info,
                 hipStream_t s, bool* all_converged, PairRec* rec);
// right-hand sides of several systems (ctxs[sys[r]]) in one persistent loop
void solve_multi(int nsys, gfcc_ctx* const* ctxs, int64_t nrhs, const int32_t* sys, const int64_t* p,
                 const double* omega, double eta, int64_t nq, const int64_t* q, const gfcc_solve_opts* opts,
                 double* G, gfcc_rhs_info* info, hipStream_t s, bool* all_converged);
// multi-shift GMRES over all frequencies of each orbital (shifts.hip)
void solve_shifts(gfcc_ctx* c, int64_t np, const int64_t* p, int64_t nw, const double* omega, double eta,
                  int64_t nq, const int64_t* q, const gfcc_shift_opts* o, double* G, double* X,
                  gfcc_rhs_info* info, hipStream_t s, bool* all_converged);

// Device-memory plan of one system (bytes): what the context keeps, what the
// caller's inputs hold, what the build needs on top, and the solver's share.
struct MemPlan {
  double input_L, input_t2, input_l2;
  double ring, ladder, wovoo, wooov, chol, rows_1h, left, vectors, small;
  double context_fp64, context_lowp;
  double build_fixed, build_chunk_min;
  double per_slot, sigma_ws, total, build_peak;
};
MemPlan plan_memory(int64_t o, int64_t v, int64_t Q, int prec, int restart, int flexible, int64_t window,
                    bool lambda_given);

// Vectors inside the library are "planes": for nb complex vectors, 2*nb planes
// of Dp doubles (re of vector 0, im of vector 0, re of vector 1, ...).
void build_intermediates(gfcc_ctx* c, const gfcc_system* sys, hipStream_t s);
void build_lowprec(gfcc_ctx* c, int which, hipStream_t s);
void sigma_planes(gfcc_ctx* c, int64_t nplanes, const double* x, double* y, gfcc_precision prec,
                  hipStream_t s);
// sigma for several systems at once (the ring GEMMs of all in grouped launches)
struct SigmaJob {
  gfcc_ctx* c;
  int64_t P;
  const double* x;
  double* y;
};
void sigma_group(const SigmaJob* jobs, int nj, gfcc_precision prec, hipStream_t s);
// interleaved complex [nb][D] <-> planes [2 nb][Dp]
void to_planes(gfcc_ctx* c, int64_t nb, const double* xi, double* planes, hipStream_t s);
void from_planes(gfcc_ctx* c, int64_t nb, const double* planes, double* xi, hipStream_t s);
// b_p (real plane) for orbitals orb_dev[0:n] in [0, o + v): e_p for occupied p,
// [a_p, T]|Phi> for virtual p; out [n][Dp]
void make_rhs_rows(gfcc_ctx* c, int64_t n, const int64_t* orb_dev, double* out, hipStream_t s);
// c_q (real plane) for orbitals orb_dev[0:n] in [0, o + v); out [n][Dp]
void make_left_rows(gfcc_ctx* c, int64_t n, const int64_t* orb_dev, double* out, hipStream_t s);
// A[k] = sgn(eta)/pi sum_p Im G[p][k] for G [np][ld] complex (device)
void spectral(int64_t np, int64_t nw, const double* G, int64_t ld, double eta, double* A, hipStream_t s);
// G[r][k] = c_{q_k} . x_r (planes), complex interleaved output
void greens_planes(gfcc_ctx* c, int64_t nb, const double* planes, int64_t nq, const int64_t* q_dev,
                   double* G, hipStream_t s);
// the same product with caller-provided left rows and split-K partials (no library buffers)
int64_t greens_part_doubles(gfcc_ctx* c, int64_t nb, int64_t nq);
void greens_rows(gfcc_ctx* c, int64_t nb, const double* planes, int64_t nq, const double* rows, double* G,
                 double* part, hipStream_t s);

// electron-attachment sector (ea.hip): blocks of Hbar_N on 1p + 2p1h, sigma on planes, and the
// rows of the linear system (-omega - i eta + Hbar_N) Y = -abar_q^+|Phi> and of G = c'_p . Y
void build_ea(gfcc_ctx* c, const gfcc_system* sys, hipStream_t s);
void ea_sigma_planes(gfcc_ctx* c, int64_t nplanes, const double* x, double* y, gfcc_precision prec, hipStream_t s);
void build_ea_lowprec(gfcc_ctx* c, hipStream_t s);
// FP16 operand scale of n doubles at x: which = 0 writes ws_vsc[0] = s, [1] = 1/s; which = 1 writes
// [2] = s_z and [3] = 1/([0] s_z) (sigma.hip)
void vector_scale(gfcc_ctx* c, const double* x, int64_t n, int which, hipStream_t s);
void ea_rhs_rows(gfcc_ctx* c, int64_t n, const int64_t* orb_dev, double* out, hipStream_t s);
void ea_left_rows(gfcc_ctx* c, int64_t n, const int64_t* orb_dev, double* out, hipStream_t s);

// open-shell IP over spin orbitals (uhf.hip)
void build_uhf(gfcc_ctx* c, const gfcc_uhf_system* sys, hipStream_t s);
void uhf_sigma_planes(gfcc_ctx* c, int64_t nplanes, const double* x, double* y, hipStream_t s);
void uhf_rhs_rows(gfcc_ctx* c, int64_t n, const int64_t* orb_dev, double* out, hipStream_t s);
void uhf_left_rows(gfcc_ctx* c, int64_t n, const int64_t* orb_dev, double* out, hipStream_t s);

// model-order reduction (mor.hip)
void mor_reset(gfcc_ctx* c);
int64_t mor_size(gfcc_ctx* c);
int64_t mor_extend(gfcc_ctx* c, int64_t nb, const double* X, double drop_tol, hipStream_t s, double* t_basis,
                   double* t_project);
void mor_model(gfcc_ctx* c, int64_t np, const int64_t* p, int64_t nq, const int64_t* q, bool diag, int64_t nw,
               const double* w, double eta, double* G, hipStream_t s);
void mor_export(gfcc_ctx* c, int which, double* dst, hipStream_t s);
void mor_greens(gfcc_ctx* c, int64_t np, const int64_t* p, int64_t nw, const double* w, double eta,
                const gfcc_mor_opts* o, double* G, int32_t* level_of, gfcc_mor_report* rep, hipStream_t s,
                bool* all_converged);

// tile autotuner (tune.hip)
void tune_load(gfcc_ctx* c, const char* path);
void tune_save(gfcc_ctx* c, const char* path);
// time every tile configuration on the sigma GEMM shapes of a P-plane batch
// (ring, hole-hole ladder, three-body + 2h1p<-1h) and keep the fastest
void tune_ring(gfcc_ctx* c, Prec p, int64_t P, hipStream_t s);
// tuned tile for a shape, else the closest tuned shape of the same precision and K, else the default
int tuned_cfg(gfcc_ctx* c, Prec p, int64_t M, int64_t N, int64_t K);

// timing helpers (no-ops when profiling is off)
void prof_begin(gfcc_ctx* c, const char* name, hipStream_t s);
void prof_end(gfcc_ctx* c, const char* name, hipStream_t s, double flops, double bytes);
void prof_collect(gfcc_ctx* c);
}  // namespace gfcc

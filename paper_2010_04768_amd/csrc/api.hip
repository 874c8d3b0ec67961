// C ABI of libgfcc (see include/gfcc.h).  Argument checking, error capture
// and dispatch to the build / sigma / solver / Green's-function code.
#include <chrono>
#include <cstddef>
#include <cmath>
#include <cstring>
#include <exception>
#include <map>
#include <mutex>
#include <string>

#include "ctx.h"

namespace gfcc {
static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }
}  // namespace gfcc

// ---------------------------------------------------------------- fixed scratch
// Device memory of the allocation-free entry points: one static array per GPU,
// held from module load until the process ends.  In host code `scratch` only
// names the symbol; its address on a device comes from hipGetSymbolAddress with
// that device current, looked up once per device when a context is built there.
namespace {
constexpr size_t kFixedScratchBytes = size_t(64) << 20;  // 64 MiB
__device__ __align__(256) unsigned char scratch[kFixedScratchBytes];

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_of_device;

void* fixed_scratch_address(int dev) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_of_device.find(dev);
  if (it != g_scratch_of_device.end()) return it->second;
  void* ptr = nullptr;
  GFCC_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  GFCC_CHECK(ptr != nullptr, GFCC_E_HIP, "hipGetSymbolAddress returned no address for the fixed scratch");
  g_scratch_of_device[dev] = ptr;
  return ptr;
}
}  // namespace

using namespace gfcc;

template <typename F>
static gfcc_status guarded(F&& f) {
  try {
    f();
    return GFCC_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.st;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return GFCC_E_OOM;
  } catch (const std::exception& e) {
    set_error(e.what());
    return GFCC_E_STATE;
  }
}

static hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

// entry points built on the ionisation sector's operands only
static void ip_sector(const gfcc_ctx* c, const char* what) {
  GFCC_CHECK(c, GFCC_E_ARG, "null context");
  GFCC_CHECK(c->sector == 0, GFCC_E_STATE,
             std::string(what) + " is not available on an electron-attachment or open-shell context");
}

extern "C" {

gfcc_status gfcc_build_intermediates(const gfcc_system* sys, void* stream, gfcc_ctx** out) {
  return guarded([&] {
    GFCC_CHECK(sys && out, GFCC_E_ARG, "null argument");
    GFCC_CHECK(sys->n_occ >= 1 && sys->n_vir >= 1 && sys->n_chol >= 1, GFCC_E_ARG,
               "n_occ, n_vir and n_chol must be >= 1");
    GFCC_CHECK(sys->n_occ <= 4096 && sys->n_vir <= 65536, GFCC_E_ARG, "dimensions out of range");
    GFCC_CHECK(sys->eps && sys->L && sys->t1 && sys->t2, GFCC_E_ARG, "eps, L, t1 and t2 are required");
    *out = nullptr;
    gfcc_ctx* c = new gfcc_ctx();
    try {
      c->o = sys->n_occ;
      c->v = sys->n_vir;
      c->Q = sys->n_chol;
      c->n = c->o + c->v;
      c->ov = c->o * c->v;
      c->oo = c->o * c->o;
      c->oov = c->oo * c->v;
      c->D = c->o + c->oov;
      c->o_pad = round_up(c->o, 8);
      c->Dp = c->o_pad + round_up(c->oov, 8);
      c->n1 = c->o;
      c->p1 = c->o_pad;
      c->n2 = c->oov;
      c->kp = round_up(c->ov, 8);
      c->k2 = 2 * c->kp;
      c->op2 = round_up(c->oo, 8);
      c->vp = round_up(c->v, 8);
      c->Qp = round_up(c->Q, 8);
      hipStream_t s = as_stream(stream);
      GFCC_HIP(hipGetDevice(&c->device));
      c->fixed_scratch = fixed_scratch_address(c->device);
      build_intermediates(c, sys, s);
      GFCC_HIP(hipStreamSynchronize(s));
    } catch (...) {
      delete c;
      throw;
    }
    *out = c;
  });
}

gfcc_status gfcc_build_ea_intermediates(const gfcc_system* sys, void* stream, gfcc_ctx** out) {
  return guarded([&] {
    GFCC_CHECK(sys && out, GFCC_E_ARG, "null argument");
    GFCC_CHECK(sys->n_occ >= 1 && sys->n_vir >= 1 && sys->n_chol >= 1, GFCC_E_ARG,
               "n_occ, n_vir and n_chol must be >= 1");
    GFCC_CHECK(sys->n_occ <= 4096 && sys->n_vir <= 4096, GFCC_E_ARG, "dimensions out of range");
    GFCC_CHECK(sys->eps && sys->L && sys->t1 && sys->t2, GFCC_E_ARG, "eps, L, t1 and t2 are required");
    *out = nullptr;
    gfcc_ctx* c = new gfcc_ctx();
    try {
      c->sector = 1;
      c->o = sys->n_occ;
      c->v = sys->n_vir;
      c->Q = sys->n_chol;
      c->n = c->o + c->v;
      c->ov = c->o * c->v;
      c->oo = c->o * c->o;
      c->oov = c->oo * c->v;
      c->n1 = c->v;
      c->p1 = round_up(c->v, 8);
      c->n2 = c->o * c->v * c->v;
      c->D = c->n1 + c->n2;
      c->Dp = c->p1 + round_up(c->n2, 8);
      c->o_pad = round_up(c->o, 8);
      c->kp = round_up(c->ov, 8);
      c->k2 = 2 * c->kp;
      c->op2 = round_up(c->oo, 8);
      c->vp = round_up(c->v, 8);
      c->Qp = round_up(c->Q, 8);
      hipStream_t s = as_stream(stream);
      GFCC_HIP(hipGetDevice(&c->device));
      c->fixed_scratch = fixed_scratch_address(c->device);
      build_ea(c, sys, s);
      GFCC_HIP(hipStreamSynchronize(s));
    } catch (...) {
      delete c;
      throw;
    }
    *out = c;
  });
}

gfcc_status gfcc_build_uhf_intermediates(const gfcc_uhf_system* sys, void* stream, gfcc_ctx** out) {
  return guarded([&] {
    GFCC_CHECK(sys && out, GFCC_E_ARG, "null argument");
    GFCC_CHECK(sys->n >= 2 && sys->n <= 2048 && sys->n_chol >= 1, GFCC_E_ARG, "bad n or n_chol");
    GFCC_CHECK(sys->n_occ_b >= 1 && sys->n_occ_b <= sys->n_occ_a && sys->n_occ_a < sys->n, GFCC_E_ARG,
               "need 1 <= n_occ_b <= n_occ_a < n");
    GFCC_CHECK(sys->eps_a && sys->eps_b && sys->La && sys->Lb && sys->t1a && sys->t1b && sys->t2aa && sys->t2ab &&
                   sys->t2bb, GFCC_E_ARG, "eps, L, t1 and t2 blocks are required");
    const bool lam = sys->l1a || sys->l1b || sys->l2aa || sys->l2ab || sys->l2bb;
    GFCC_CHECK(!lam || (sys->l1a && sys->l1b && sys->l2aa && sys->l2ab && sys->l2bb), GFCC_E_ARG,
               "give every Lambda block or none");
    *out = nullptr;
    gfcc_ctx* c = new gfcc_ctx();
    try {
      c->sector = 2;
      c->o = sys->n_occ_a + sys->n_occ_b;
      c->v = 2 * sys->n - c->o;
      c->Q = sys->n_chol;
      c->n = c->o + c->v;
      c->ov = c->o * c->v;
      c->oo = c->o * c->o;
      c->oov = c->oo * c->v;
      c->o_pad = round_up(c->o, 8);
      c->n1 = c->o;
      c->p1 = c->o_pad;
      c->n2 = c->oov;
      c->D = c->n1 + c->n2;
      c->Dp = c->p1 + round_up(c->n2, 8);
      c->kp = round_up(c->ov, 8);
      c->k2 = 2 * c->kp;
      c->op2 = round_up(c->oo, 8);
      c->vp = round_up(c->v, 8);
      c->Qp = round_up(c->Q, 8);
      hipStream_t s = as_stream(stream);
      GFCC_HIP(hipGetDevice(&c->device));
      c->fixed_scratch = fixed_scratch_address(c->device);
      build_uhf(c, sys, s);
      GFCC_HIP(hipStreamSynchronize(s));
    } catch (...) {
      delete c;
      throw;
    }
    *out = c;
  });
}

gfcc_status gfcc_plan_memory(int64_t n_occ, int64_t n_vir, int64_t n_chol, gfcc_precision prec, int32_t restart,
                             int32_t flexible, int64_t window, int32_t lambda_given, gfcc_memory_plan* out) {
  return guarded([&] {
    GFCC_CHECK(out && out->struct_size >= sizeof(gfcc_memory_plan), GFCC_E_ARG, "bad plan struct");
    GFCC_CHECK(n_occ >= 1 && n_vir >= 1 && n_chol >= 1 && window >= 0 && restart >= 1, GFCC_E_ARG, "bad sizes");
    GFCC_CHECK(prec >= GFCC_FP64 && prec <= GFCC_FP16_IR, GFCC_E_ARG, "bad precision");
    const MemPlan p = plan_memory(n_occ, n_vir, n_chol, prec, restart, flexible, window, lambda_given != 0);
    const size_t ss = out->struct_size;
    *out = gfcc_memory_plan{};
    out->struct_size = ss;
    out->input_L = p.input_L;
    out->input_t2 = p.input_t2;
    out->input_l2 = p.input_l2;
    out->ring = p.ring;
    out->ladder = p.ladder;
    out->wovoo = p.wovoo;
    out->wooov = p.wooov;
    out->cholesky = p.chol;
    out->rows_1h = p.rows_1h;
    out->left = p.left;
    out->vectors = p.vectors;
    out->small = p.small;
    out->context_fp64 = p.context_fp64;
    out->context_lowp = p.context_lowp;
    out->build_fixed = p.build_fixed;
    out->build_chunk_min = p.build_chunk_min;
    out->per_slot = p.per_slot;
    out->sigma_workspace = p.sigma_ws;
    out->total = p.total;
    out->build_peak = p.build_peak;
  });
}

gfcc_status gfcc_dims(const gfcc_ctx* c, int64_t* D, int64_t* n_occ, int64_t* n_vir) {
  return guarded([&] {
    GFCC_CHECK(c, GFCC_E_ARG, "null context");
    if (D) *D = c->D;
    if (n_occ) *n_occ = c->o;
    if (n_vir) *n_vir = c->v;
  });
}

gfcc_status gfcc_export(gfcc_ctx* c, gfcc_block which, double* dst, void* stream) {
  return guarded([&] {
    GFCC_CHECK(c && dst, GFCC_E_ARG, "null argument");
    GFCC_CHECK(c->sector == 0 || which == GFCC_FOO || which == GFCC_FVV || which == GFCC_FOV || which == GFCC_DIAG,
               GFCC_E_STATE, "an electron-attachment or open-shell context exports FOO, FVV, FOV and DIAG only");
    hipStream_t s = as_stream(stream);
    const int64_t o = c->o, v = c->v, kp = c->kp, k2 = c->k2;
    const int id4[4] = {0, 1, 2, 3};
    auto copy = [&](const DBuf& b, int64_t n) {
      GFCC_HIP(hipMemcpyAsync(dst, b.p, size_t(n) * 8, hipMemcpyDeviceToDevice, s));
    };
    switch (which) {
      case GFCC_FOO: copy(c->Foo, o * o); break;
      case GFCC_FVV: copy(c->Fvv, v * v); break;
      case GFCC_FOV: copy(c->Fov, o * v); break;
      case GFCC_WOOOO: {  // W4T[(i,j)][(m,n)] -> [m][n][i][j]
        const int64_t op2 = c->op2;
        TView in = tview_s(c->W4T.as<double>(), {o, o, o, o}, {o, 1, o * op2, op2});
        permute(in, id4, 1.0, tview(dst, {o, o, o, o}), 0.0, s);
        break;
      }
      case GFCC_WOOOV: copy(c->Wooov, o * o * o * v); break;
      case GFCC_WOVOO: {  // WovooT[(i,j,a)][m] -> [m][a][i][j]
        const int64_t op = c->o_pad;
        TView in = tview_s(c->WovooT.as<double>(), {o, v, o, o}, {1, op, o * v * op, v * op});
        permute(in, id4, 1.0, tview(dst, {o, v, o, o}), 0.0, s);
        break;
      }
      case GFCC_WOVVO: {  // WW[(j,a)][(m,e)] -> [m][a][e][j]
        TView in = tview_s(c->WW.as<double>(), {o, v, v, o}, {v, k2, 1, v * k2});
        permute(in, id4, 1.0, tview(dst, {o, v, v, o}), 0.0, s);
        break;
      }
      case GFCC_WOVOV: {  // WW[(j,a)][kp + (m,e)] -> [m][a][j][e], without the folded one-body terms
        TView in = tview_s(c->WW.as<double>() + kp, {o, v, o, v}, {v, k2, v * k2, 1});
        permute(in, id4, 1.0, tview(dst, {o, v, o, v}), 0.0, s);
        // remove  Foo_off[m,j] d_ae
        const int id3[3] = {0, 1, 2}, id2[2] = {0, 1};
        const double* Foo = c->Foo.as<double>();
        const double* Fvv = c->Fvv.as<double>();
        TView foo_b = tview_s(const_cast<double*>(Foo), {o, v, o}, {1, 0, o});  // [j][a][m] -> Foo[m][j]
        TView foo_d = tview_s(const_cast<double*>(Foo), {o, v}, {o + 1, 0});    // [j][a]    -> Foo[j][j]
        TView o_ae = tview_s(dst, {o, v, o}, {v, o * v + 1, v * o * v});        // [j][a][m] at [m][a][j][a]
        TView o_d = tview_s(dst, {o, v}, {v * o * v + v, o * v + 1});            // m = j, e = a
        permute(foo_b, id3, -1.0, o_ae, 1.0, s);
        permute(foo_d, id2, 1.0, o_d, 1.0, s);
        // remove -1/2 Fvv_off[a,e] d_jm
        TView fvv_b = tview_s(const_cast<double*>(Fvv), {o, v, v}, {0, v, 1});  // [j][a][e] -> Fvv[a][e]
        TView fvv_d = tview_s(const_cast<double*>(Fvv), {o, v}, {0, v + 1});    // [j][a]    -> Fvv[a][a]
        TView o_jm = tview_s(dst, {o, v, v}, {v * o * v + v, o * v, 1});        // [j][a][e] at [j][a][j][e]
        permute(fvv_b, id3, 0.5, o_jm, 1.0, s);
        permute(fvv_d, id2, -0.5, o_d, 1.0, s);
        break;
      }
      case GFCC_DIAG:
        GFCC_HIP(hipMemcpyAsync(dst, c->diag.p, size_t(c->n1) * 8, hipMemcpyDeviceToDevice, s));
        GFCC_HIP(hipMemcpyAsync(dst + c->n1, c->diag.as<double>() + c->p1, size_t(c->n2) * 8,
                                hipMemcpyDeviceToDevice, s));
        break;
      case GFCC_LEFT:
        GFCC_HIP(hipMemcpy2DAsync(dst, size_t(c->D) * 8, c->left.p, size_t(c->Dp) * 8, size_t(o) * 8, size_t(o),
                                  hipMemcpyDeviceToDevice, s));
        GFCC_HIP(hipMemcpy2DAsync(dst + o, size_t(c->D) * 8, c->left.as<double>() + c->o_pad, size_t(c->Dp) * 8,
                                  size_t(c->oov) * 8, size_t(o), hipMemcpyDeviceToDevice, s));
        break;
      default: throw Error{GFCC_E_ARG, "unknown block"};
    }
  });
}

gfcc_status gfcc_sigma(gfcc_ctx* c, int64_t nrhs, const double* X, double* Y, gfcc_precision prec, void* stream) {
  return guarded([&] {
    GFCC_CHECK(c, GFCC_E_ARG, "null context");
    GFCC_CHECK(nrhs >= 0, GFCC_E_ARG, "nrhs < 0");
    GFCC_CHECK(prec >= GFCC_FP64 && prec <= GFCC_FP16_IR, GFCC_E_ARG, "bad precision");
    GFCC_CHECK(c->sector == 0 || prec == GFCC_FP64 || (c->sector == 1 && prec == GFCC_FP16_IR), GFCC_E_ARG,
               "the electron-attachment sigma runs in FP64 or FP16, the open-shell sigma in FP64");
    if (nrhs == 0) return;
    GFCC_CHECK(X && Y && X != Y, GFCC_E_ARG, "X and Y must be distinct device buffers");
    hipStream_t s = as_stream(stream);
    const int64_t chunk = 64;
    for (int64_t r0 = 0; r0 < nrhs; r0 += chunk) {
      const int64_t nb = std::min(chunk, nrhs - r0);
      c->ws_in.ensure(size_t(2 * nb * c->Dp) * 8, s);
      c->ws_out.ensure(size_t(2 * nb * c->Dp) * 8, s);
      to_planes(c, nb, X + r0 * c->D * 2, c->ws_in.as<double>(), s);
      sigma_planes(c, 2 * nb, c->ws_in.as<double>(), c->ws_out.as<double>(), prec, s);
      from_planes(c, nb, c->ws_out.as<double>(), Y + r0 * c->D * 2, s);
    }
  });
}

gfcc_status gfcc_spectral(int64_t np, int64_t n_omega, const double* G, int64_t ld, double eta, double* A,
                          void* stream) {
  return guarded([&] {
    GFCC_CHECK(np >= 0 && n_omega >= 0 && ld >= n_omega, GFCC_E_ARG, "bad sizes (need ld >= n_omega)");
    if (n_omega == 0) return;
    GFCC_CHECK(A && (G || np == 0), GFCC_E_ARG, "null argument");
    GFCC_CHECK(std::isfinite(eta) && eta != 0.0, GFCC_E_ARG, "eta must be finite and non-zero");
    spectral(np, n_omega, G, ld, eta, A, as_stream(stream));
  });
}

gfcc_status gfcc_greens(gfcc_ctx* c, int64_t nrhs, const int64_t* p, const double* X, int64_t nq,
                        const int64_t* q, double* G, void* stream) {
  return guarded([&] {
    GFCC_CHECK(c, GFCC_E_ARG, "null context");
    GFCC_CHECK(nrhs >= 0 && nq >= 0, GFCC_E_ARG, "negative size");
    if (nrhs == 0 || nq == 0) return;
    GFCC_CHECK(X && G, GFCC_E_ARG, "null argument");
    GFCC_CHECK(q != nullptr || (nq == 1 && p != nullptr), GFCC_E_ARG, "q == NULL requires nq == 1 and p");
    const int64_t norb = c->o + c->v;
    if (q)
      for (int64_t k = 0; k < nq; ++k) GFCC_CHECK(q[k] >= 0 && q[k] < norb, GFCC_E_ARG, "q out of range");
    else
      for (int64_t r = 0; r < nrhs; ++r) GFCC_CHECK(p[r] >= 0 && p[r] < norb, GFCC_E_ARG, "p out of range");
    hipStream_t s = as_stream(stream);
    // q list (shared by every vector), or the diagonal form's own orbital per vector
    const int64_t nlist = q ? nq : nrhs;
    DBuf qd;
    qd.ensure(size_t(nlist) * 8, s);
    GFCC_HIP(hipMemcpyAsync(qd.p, q ? q : p, size_t(nlist) * 8, hipMemcpyHostToDevice, s));
    const int64_t chunk = 64;
    for (int64_t r0 = 0; r0 < nrhs; r0 += chunk) {
      const int64_t nb = std::min(chunk, nrhs - r0);
      c->ws_in.ensure(size_t(2 * nb * c->Dp) * 8, s);
      to_planes(c, nb, X + r0 * c->D * 2, c->ws_in.as<double>(), s);
      if (q) {
        greens_planes(c, nb, c->ws_in.as<double>(), nq, qd.as<int64_t>(), G + r0 * nq * 2, s);
      } else {
        for (int64_t b = 0; b < nb; ++b)
          greens_planes(c, 1, c->ws_in.as<double>() + 2 * b * c->Dp, 1, qd.as<int64_t>() + r0 + b,
                        G + (r0 + b) * 2, s);
      }
    }
    GFCC_HIP(hipStreamSynchronize(s));  // qd and the host lists are released on return
  });
}

// gfcc_greens without any device allocation: the vectors' planes, the left rows, the
// orbital list and the split-K partials live in the fixed scratch array.
gfcc_status gfcc_greens_noalloc(gfcc_ctx* c, int64_t nrhs, const int64_t* p, const double* X, int64_t nq,
                                const int64_t* q, double* G, void* stream) {
  return guarded([&] {
    GFCC_CHECK(c, GFCC_E_ARG, "null context");
    GFCC_CHECK(nrhs >= 0 && nq >= 0, GFCC_E_ARG, "negative size");
    if (nrhs == 0 || nq == 0) return;
    GFCC_CHECK(X && G, GFCC_E_ARG, "null argument");
    GFCC_CHECK(q != nullptr || (nq == 1 && p != nullptr), GFCC_E_ARG, "q == NULL requires nq == 1 and p");
    const int64_t norb = c->o + c->v;
    if (q)
      for (int64_t k = 0; k < nq; ++k) GFCC_CHECK(q[k] >= 0 && q[k] < norb, GFCC_E_ARG, "q out of range");
    else
      for (int64_t r = 0; r < nrhs; ++r) GFCC_CHECK(p[r] >= 0 && p[r] < norb, GFCC_E_ARG, "p out of range");
    int dev = -1;
    GFCC_HIP(hipGetDevice(&dev));
    GFCC_CHECK(dev == c->device && c->fixed_scratch, GFCC_E_STATE,
               "the context's device must be current for the allocation-free entry points");
    hipStream_t s = as_stream(stream);
    const int64_t Dp = c->Dp;
    const size_t plane = size_t(Dp) * 8;
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    // regions: orbital list | left rows | planes of nb vectors | split-K partials
    const int64_t nrows = q ? nq : 1;   // the diagonal form takes one vector (and row) at a time
    const int64_t nlist = q ? nq : 1;
    const size_t list_b = up(size_t(nlist) * 8), rows_b = up(size_t(nrows) * plane);
    auto need = [&](int64_t nb) {
      return list_b + rows_b + up(size_t(2 * nb) * plane) + up(size_t(greens_part_doubles(c, nb, nrows)) * 8);
    };
    int64_t nb = q ? std::min<int64_t>(nrhs, 64) : 1;
    while (nb > 1 && need(nb) > kFixedScratchBytes) --nb;
    GFCC_CHECK(need(nb) <= kFixedScratchBytes, GFCC_E_ARG,
               "request exceeds the fixed scratch of the allocation-free entry point: " +
                   std::to_string(need(nb)) + " bytes needed, " + std::to_string(kFixedScratchBytes) + " available");
    unsigned char* base = static_cast<unsigned char*>(c->fixed_scratch);
    int64_t* list = reinterpret_cast<int64_t*>(base);
    double* rows = reinterpret_cast<double*>(base + list_b);
    double* planes = reinterpret_cast<double*>(base + list_b + rows_b);
    double* part = reinterpret_cast<double*>(base + list_b + rows_b + up(size_t(2 * nb) * plane));
    if (q) {
      GFCC_HIP(hipMemcpyAsync(list, q, size_t(nq) * 8, hipMemcpyHostToDevice, s));
      make_left_rows(c, nq, list, rows, s);
    }
    for (int64_t r0 = 0; r0 < nrhs; r0 += nb) {
      const int64_t n = std::min(nb, nrhs - r0);
      if (!q) {
        GFCC_HIP(hipMemcpyAsync(list, p + r0, 8, hipMemcpyHostToDevice, s));
        make_left_rows(c, 1, list, rows, s);
      }
      // the planes' padding must read as zero: the array keeps the previous call's contents
      GFCC_HIP(hipMemsetAsync(planes, 0, size_t(2 * n) * plane, s));
      to_planes(c, n, X + r0 * c->D * 2, planes, s);
      greens_rows(c, n, planes, nrows, rows, G + r0 * nq * 2, part, s);
    }
    GFCC_HIP(hipStreamSynchronize(s));  // the host lists are only read by the copies above
  });
}

gfcc_status gfcc_solve_batch(gfcc_ctx* c, int64_t nrhs, const int64_t* p, const double* omega, double eta,
                             int64_t nq, const int64_t* q, const gfcc_solve_opts* opts, double* G, double* X,
                             gfcc_rhs_info* info, void* stream) {
  bool all_conv = true;
  gfcc_status st = guarded([&] {
    GFCC_CHECK(c, GFCC_E_ARG, "null context");
    GFCC_CHECK(opts && opts->struct_size >= sizeof(gfcc_solve_opts), GFCC_E_ARG, "bad options struct");
    GFCC_CHECK(nrhs >= 0, GFCC_E_ARG, "nrhs < 0");
    if (nrhs == 0) return;
    GFCC_CHECK(p && omega && G && info, GFCC_E_ARG, "null argument");
    GFCC_CHECK(q != nullptr || nq == 1, GFCC_E_ARG, "q == NULL requires nq == 1");
    GFCC_CHECK(nq >= 1, GFCC_E_ARG, "nq < 1");
    for (int64_t r = 0; r < nrhs; ++r) GFCC_CHECK(p[r] >= 0 && p[r] < c->o + c->v, GFCC_E_ARG, "p out of range");
    for (int64_t r = 0; r < nrhs; ++r) GFCC_CHECK(std::isfinite(omega[r]), GFCC_E_ARG, "non-finite omega");
    GFCC_CHECK(std::isfinite(eta), GFCC_E_ARG, "non-finite eta");
    if (q)
      for (int64_t k = 0; k < nq; ++k) GFCC_CHECK(q[k] >= 0 && q[k] < c->o + c->v, GFCC_E_ARG, "q out of range");
    GFCC_CHECK(opts->tol > 0.0 && opts->restart >= 1 && opts->max_iter >= 1, GFCC_E_ARG, "bad tolerance/restart/max_iter");
    GFCC_CHECK(opts->precond >= GFCC_PC_NONE && opts->precond <= GFCC_PC_MLP, GFCC_E_ARG, "bad preconditioner");
    GFCC_CHECK(opts->precision >= GFCC_FP64 && opts->precision <= GFCC_FP16_IR, GFCC_E_ARG, "bad precision");
    GFCC_CHECK(opts->sync_every >= 0, GFCC_E_ARG, "sync_every < 0");
    if (c->sector != 0) {
      GFCC_CHECK(opts->precision == GFCC_FP64 || (c->sector == 1 && opts->precision == GFCC_FP16_IR), GFCC_E_ARG,
                 "the electron-attachment solve runs in FP64 or FP16-IR, the open-shell solve in FP64");
      GFCC_CHECK(opts->precond != GFCC_PC_MLP, GFCC_E_STATE,
                 "the learned preconditioner is trained on the closed-shell ionisation sector only");
    }
    if (c->sector == 1) {
      // (omega - Hbar_N + i eta) Y = abar^+|Phi>  is solved as  (-omega - i eta + Hbar_N) Y = -abar^+|Phi>
      std::vector<double> wneg(static_cast<size_t>(nrhs));
      for (int64_t r = 0; r < nrhs; ++r) wneg[size_t(r)] = -omega[r];
      solve_batch(c, nrhs, p, wneg.data(), eta, nq, q, opts, G, X, info, as_stream(stream), &all_conv, nullptr);
      return;
    }
    solve_batch(c, nrhs, p, omega, eta, nq, q, opts, G, X, info, as_stream(stream), &all_conv, nullptr);
  });
  if (st == GFCC_OK && !all_conv) return GFCC_W_NOCONV;
  return st;
}

// ---------------------------------------------------------------- learned preconditioner

static double diag_mean_abs(gfcc_ctx* c, hipStream_t s) {
  std::vector<double> h(size_t(c->Dp));
  GFCC_HIP(hipMemcpyAsync(h.data(), c->diag.p, size_t(c->Dp) * 8, hipMemcpyDeviceToHost, s));
  GFCC_HIP(hipStreamSynchronize(s));
  double acc = 0.0;
  for (int64_t i = 0; i < c->o; ++i) acc += std::fabs(h[size_t(i)]);
  for (int64_t i = 0; i < c->oov; ++i) acc += std::fabs(h[size_t(c->o_pad + i)]);
  return acc / double(c->D);
}

__global__ void rms_kernel(const double* __restrict__ planes, int64_t Dp, int64_t D, double* out) {
  __shared__ double red[256];
  const double* x = planes + int64_t(blockIdx.x) * 2 * Dp;
  double acc = 0.0;
  for (int64_t t = threadIdx.x; t < 2 * Dp; t += 256) acc += x[t] * x[t];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = sqrt(red[0] / double(D));
}

gfcc_status gfcc_mlp_set_weights(gfcc_ctx* c, int32_t width, const double* params, void* stream) {
  return guarded([&] {
    ip_sector(c, "gfcc_mlp_set_weights");
    GFCC_CHECK(c && params, GFCC_E_ARG, "null argument");
    hipStream_t s = as_stream(stream);
    mlp_init(c, width, 0, s);
    c->mlp->sD = diag_mean_abs(c, s);
    GFCC_HIP(hipMemcpyAsync(c->mlp->params.p, params, size_t(mlp_n_params(width)) * 8, hipMemcpyDeviceToDevice, s));
    mlp_prepare_inference(c, s);
    GFCC_HIP(hipStreamSynchronize(s));
  });
}

gfcc_status gfcc_mlp_get_weights(gfcc_ctx* c, int32_t* width, double* params, void* stream) {
  return guarded([&] {
    ip_sector(c, "gfcc_mlp_get_weights");
    GFCC_CHECK(c && width, GFCC_E_ARG, "null argument");
    GFCC_CHECK(c->mlp != nullptr, GFCC_E_STATE, "no network in this context");
    *width = c->mlp->width;
    if (params)
      GFCC_HIP(hipMemcpyAsync(params, c->mlp->params.p, size_t(mlp_n_params(c->mlp->width)) * 8,
                              hipMemcpyDeviceToDevice, as_stream(stream)));
  });
}

gfcc_status gfcc_mlp_adam_step(gfcc_ctx* c, const double* grad, double lr, void* stream) {
  return guarded([&] {
    ip_sector(c, "gfcc_mlp_adam_step");
    GFCC_CHECK(c && grad, GFCC_E_ARG, "null argument");
    GFCC_CHECK(std::isfinite(lr) && lr > 0.0, GFCC_E_ARG, "lr must be finite and positive");
    GFCC_CHECK(c->mlp != nullptr, GFCC_E_STATE, "no network in this context");
    hipStream_t s = as_stream(stream);
    mlp_adam(c, grad, lr, s);
    mlp_prepare_inference(c, s);
    GFCC_HIP(hipStreamSynchronize(s));
  });
}

gfcc_status gfcc_mlp_forward(gfcc_ctx* c, int64_t n, const double* X, double* Y, void* stream) {
  return guarded([&] {
    ip_sector(c, "gfcc_mlp_forward");
    GFCC_CHECK(c && X && Y && n >= 0, GFCC_E_ARG, "bad argument");
    GFCC_CHECK(c->mlp != nullptr, GFCC_E_STATE, "no network in this context");
    if (n == 0) return;
    hipStream_t s = as_stream(stream);
    const int W = c->mlp->width;
    double* H1 = c->mlp->ws.get(6, n * W, s);
    double* H2 = c->mlp->ws.get(7, n * W, s);
    mlp_forward64(c, n, X, H1, H2, Y, s);
    GFCC_HIP(hipStreamSynchronize(s));
  });
}

gfcc_status gfcc_mlp_loss_grad(gfcc_ctx* c, int64_t n, const double* X, const double* T, double* loss, double* grad,
                               void* stream) {
  return guarded([&] {
    ip_sector(c, "gfcc_mlp_loss_grad");
    GFCC_CHECK(c && X && T && loss && grad && n > 0, GFCC_E_ARG, "bad argument");
    GFCC_CHECK(c->mlp != nullptr, GFCC_E_STATE, "no network in this context");
    hipStream_t s = as_stream(stream);
    mlp_loss_grad64(c, n, X, T, loss, grad, s);
    GFCC_HIP(hipStreamSynchronize(s));
  });
}

gfcc_status gfcc_mlp_features(gfcc_ctx* c, int64_t nvec, const double* R, const double* omega, double eta, double* X,
                              void* stream) {
  return guarded([&] {
    ip_sector(c, "gfcc_mlp_features");
    GFCC_CHECK(c && R && omega && X && nvec >= 0, GFCC_E_ARG, "bad argument");
    if (nvec == 0) return;
    hipStream_t s = as_stream(stream);
    if (!c->mlp) mlp_init(c, 64, 0, s);
    c->mlp->sD = diag_mean_abs(c, s);
    DBuf pl, om, nr;
    pl.ensure(size_t(2 * nvec * c->Dp) * 8, s);
    om.ensure(size_t(nvec) * 8, s);
    nr.ensure(size_t(nvec) * 8, s);
    GFCC_HIP(hipMemcpyAsync(om.p, omega, size_t(nvec) * 8, hipMemcpyHostToDevice, s));
    to_planes(c, nvec, R, pl.as<double>(), s);
    hipLaunchKernelGGL(rms_kernel, dim3(unsigned(nvec)), dim3(256), 0, s, pl.as<double>(), c->Dp, c->D, nr.as<double>());
    mlp_features(c, nvec, pl.as<double>(), om.as<double>(), nr.as<double>(), eta, X, s);
    GFCC_HIP(hipStreamSynchronize(s));
  });
}

gfcc_status gfcc_mlp_apply(gfcc_ctx* c, int64_t nvec, const double* R, const double* omega, double eta, double* U,
                           void* stream) {
  return guarded([&] {
    ip_sector(c, "gfcc_mlp_apply");
    GFCC_CHECK(c && R && omega && U && nvec >= 0, GFCC_E_ARG, "bad argument");
    GFCC_CHECK(c->mlp && c->mlp->trained, GFCC_E_STATE, "no trained network in this context");
    if (nvec == 0) return;
    hipStream_t s = as_stream(stream);
    DBuf pl, out, om, nr;
    pl.ensure(size_t(2 * nvec * c->Dp) * 8, s);
    out.ensure(size_t(2 * nvec * c->Dp) * 8, s);
    om.ensure(size_t(nvec) * 8, s);
    nr.ensure(size_t(nvec) * 8, s);
    GFCC_HIP(hipMemcpyAsync(om.p, omega, size_t(nvec) * 8, hipMemcpyHostToDevice, s));
    to_planes(c, nvec, R, pl.as<double>(), s);
    hipLaunchKernelGGL(rms_kernel, dim3(unsigned(nvec)), dim3(256), 0, s, pl.as<double>(), c->Dp, c->D, nr.as<double>());
    MlpApplyArgs a;
    a.src = pl.as<double>();
    a.omega = om.as<double>();
    a.nrm = nr.as<double>();
    a.eta = eta;
    a.dst = out.as<double>();
    mlp_apply(c, a, nvec, s);
    from_planes(c, nvec, out.as<double>(), U, s);
    GFCC_HIP(hipStreamSynchronize(s));
  });
}

gfcc_status gfcc_solve_multi(int32_t nsys, gfcc_ctx* const* ctxs, int64_t nrhs, const int32_t* sys,
                             const int64_t* p, const double* omega, double eta, int64_t nq, const int64_t* q,
                             const gfcc_solve_opts* opts, double* G, gfcc_rhs_info* info, void* stream) {
  bool all_conv = true;
  gfcc_status st = guarded([&] {
    GFCC_CHECK(nsys >= 1 && nsys <= 16 && ctxs, GFCC_E_ARG, "nsys must be in [1, 16]");
    for (int k = 0; k < nsys; ++k) {
      ip_sector(ctxs[k], "gfcc_solve_multi");
      for (int j = 0; j < k; ++j) GFCC_CHECK(ctxs[j] != ctxs[k], GFCC_E_ARG, "a context appears twice");
    }
    GFCC_CHECK(opts && opts->struct_size >= sizeof(gfcc_solve_opts), GFCC_E_ARG, "bad options struct");
    GFCC_CHECK(nrhs >= 0, GFCC_E_ARG, "nrhs < 0");
    if (nrhs == 0) return;
    GFCC_CHECK(sys && p && omega && G && info, GFCC_E_ARG, "null argument");
    GFCC_CHECK(q != nullptr || nq == 1, GFCC_E_ARG, "q == NULL requires nq == 1");
    GFCC_CHECK(nq >= 1, GFCC_E_ARG, "nq < 1");
    for (int64_t r = 0; r < nrhs; ++r) {
      GFCC_CHECK(sys[r] >= 0 && sys[r] < nsys, GFCC_E_ARG, "system index out of range");
      const gfcc_ctx* c = ctxs[sys[r]];
      GFCC_CHECK(p[r] >= 0 && p[r] < c->o + c->v, GFCC_E_ARG, "p out of range");
      GFCC_CHECK(std::isfinite(omega[r]), GFCC_E_ARG, "non-finite omega");
    }
    GFCC_CHECK(std::isfinite(eta), GFCC_E_ARG, "non-finite eta");
    if (q)
      for (int k = 0; k < nsys; ++k)
        for (int64_t j = 0; j < nq; ++j)
          GFCC_CHECK(q[j] >= 0 && q[j] < ctxs[k]->o + ctxs[k]->v, GFCC_E_ARG, "q out of range for a system");
    GFCC_CHECK(opts->tol > 0.0 && opts->restart >= 1 && opts->max_iter >= 1, GFCC_E_ARG, "bad tolerance/restart/max_iter");
    GFCC_CHECK(opts->precond >= GFCC_PC_NONE && opts->precond <= GFCC_PC_MLP, GFCC_E_ARG, "bad preconditioner");
    GFCC_CHECK(opts->precision >= GFCC_FP64 && opts->precision <= GFCC_FP16_IR, GFCC_E_ARG, "bad precision");
    GFCC_CHECK(opts->sync_every >= 0, GFCC_E_ARG, "sync_every < 0");
    if (opts->precond == GFCC_PC_MLP)
      for (int k = 0; k < nsys; ++k)
        GFCC_CHECK(ctxs[k]->mlp && ctxs[k]->mlp->trained, GFCC_E_STATE,
                   "GFCC_PC_MLP needs trained or loaded network weights on every system");
    solve_multi(nsys, ctxs, nrhs, sys, p, omega, eta, nq, q, opts, G, info, as_stream(stream), &all_conv);
  });
  if (st == GFCC_OK && !all_conv) return GFCC_W_NOCONV;
  return st;
}

gfcc_status gfcc_solve_shifts(gfcc_ctx* c, int64_t np, const int64_t* p, int64_t n_omega, const double* omega,
                              double eta, int64_t nq, const int64_t* q, const gfcc_shift_opts* opts, double* G,
                              double* X, gfcc_rhs_info* info, void* stream) {
  bool all_conv = true;
  gfcc_status st = guarded([&] {
    GFCC_CHECK(c, GFCC_E_ARG, "null context");
    GFCC_CHECK(opts && opts->struct_size >= sizeof(gfcc_shift_opts), GFCC_E_ARG, "bad options struct");
    GFCC_CHECK(np >= 0 && n_omega >= 0, GFCC_E_ARG, "negative size");
    if (np == 0 || n_omega == 0) return;
    GFCC_CHECK(p && omega && G && info, GFCC_E_ARG, "null argument");
    GFCC_CHECK(q != nullptr || nq == 1, GFCC_E_ARG, "q == NULL requires nq == 1");
    GFCC_CHECK(nq >= 1, GFCC_E_ARG, "nq < 1");
    for (int64_t r = 0; r < np; ++r) GFCC_CHECK(p[r] >= 0 && p[r] < c->o + c->v, GFCC_E_ARG, "p out of range");
    if (q)
      for (int64_t k = 0; k < nq; ++k) GFCC_CHECK(q[k] >= 0 && q[k] < c->o + c->v, GFCC_E_ARG, "q out of range");
    for (int64_t k = 0; k < n_omega; ++k) GFCC_CHECK(std::isfinite(omega[k]), GFCC_E_ARG, "non-finite omega");
    GFCC_CHECK(std::isfinite(eta), GFCC_E_ARG, "non-finite eta");
    GFCC_CHECK(opts->tol > 0.0 && opts->max_dim >= 0 && opts->max_dim <= 512 && opts->batch >= 0, GFCC_E_ARG,
               "bad tol / max_dim / batch");
    if (opts->use_fallback) {
      const gfcc_solve_opts& f = opts->fallback;
      GFCC_CHECK(f.struct_size >= sizeof(gfcc_solve_opts), GFCC_E_ARG, "bad fallback options struct");
      GFCC_CHECK(f.tol > 0.0 && f.restart >= 1 && f.max_iter >= 1, GFCC_E_ARG, "bad fallback tolerance/restart/max_iter");
      GFCC_CHECK(f.precond >= GFCC_PC_NONE && f.precond <= GFCC_PC_MLP, GFCC_E_ARG, "bad fallback preconditioner");
      GFCC_CHECK(f.precision >= GFCC_FP64 && f.precision <= GFCC_FP16_IR, GFCC_E_ARG, "bad fallback precision");
      GFCC_CHECK(c->sector == 0 ||
                     ((f.precision == GFCC_FP64 || (c->sector == 1 && f.precision == GFCC_FP16_IR)) &&
                      f.precond != GFCC_PC_MLP),
                 GFCC_E_ARG,
                 "the fallback of an electron-attachment context is FP64 or FP16-IR, of an open-shell context FP64, "
                 "both without the network");
    }
    if (c->sector == 1) {  // the EA system (omega - Hbar_N + i eta) Y = b' as (-omega - i eta + Hbar_N) Y = -b'
      std::vector<double> wneg(static_cast<size_t>(n_omega));
      for (int64_t k = 0; k < n_omega; ++k) wneg[size_t(k)] = -omega[k];
      solve_shifts(c, np, p, n_omega, wneg.data(), eta, nq, q, opts, G, X, info, as_stream(stream), &all_conv);
      return;
    }
    solve_shifts(c, np, p, n_omega, omega, eta, nq, q, opts, G, X, info, as_stream(stream), &all_conv);
  });
  if (st == GFCC_OK && !all_conv) return GFCC_W_NOCONV;
  return st;
}

gfcc_status gfcc_mlp_train(gfcc_ctx* c, int64_t nrhs, const int64_t* p, const double* omega, double eta,
                           const gfcc_mlp_opts* mo, gfcc_mlp_report* rep, void* stream) {
  return guarded([&] {
    ip_sector(c, "gfcc_mlp_train");
    GFCC_CHECK(c && p && omega && mo && nrhs > 0, GFCC_E_ARG, "bad argument");
    GFCC_CHECK(mo->struct_size >= sizeof(gfcc_mlp_opts), GFCC_E_ARG, "bad options struct");
    GFCC_CHECK(mo->steps >= 0 && mo->batch >= 1 && mo->pair_restart >= 1 && mo->max_pairs >= 1 && mo->lr > 0.0,
               GFCC_E_ARG, "bad training options");
    for (int64_t r = 0; r < nrhs; ++r) GFCC_CHECK(p[r] >= 0 && p[r] < c->o + c->v, GFCC_E_ARG, "p out of range");
    hipStream_t s = as_stream(stream);
    const auto t0 = std::chrono::steady_clock::now();
    mlp_init(c, mo->width, mo->seed, s);
    c->mlp->sD = diag_mean_abs(c, s);
    // 1. pairs from FP64 Jacobi solves
    const int64_t Dp = c->Dp;
    DBuf bR, bX, bXs, bE, bG;
    bR.ensure(size_t(mo->max_pairs) * 2 * Dp * 8, s);
    bX.ensure(size_t(mo->max_pairs) * 2 * Dp * 8, s);
    bXs.ensure(size_t(nrhs) * 2 * Dp * 8, s);
    bG.ensure(size_t(nrhs) * 16, s);
    PairRec rec;
    rec.R = bR.as<double>();
    rec.X = bX.as<double>();
    rec.xstar = bXs.as<double>();
    rec.cap = mo->max_pairs;
    gfcc_solve_opts so{};
    so.struct_size = sizeof(so);
    so.tol = mo->data_tol > 0.0 ? mo->data_tol : 1e-11;
    so.restart = mo->pair_restart;
    so.max_iter = mo->data_max_iter > 0 ? mo->data_max_iter : 4000;
    so.precond = GFCC_PC_JACOBI;
    GFCC_CHECK(mo->data_precision >= GFCC_FP64 && mo->data_precision <= GFCC_FP16_IR, GFCC_E_ARG,
               "bad data_precision");
    so.precision = static_cast<gfcc_precision>(mo->data_precision);
    std::vector<gfcc_rhs_info> inf(static_cast<size_t>(nrhs));
    bool conv = true;
    solve_batch(c, nrhs, p, omega, eta, 1, nullptr, &so, bG.as<double>(), nullptr, inf.data(), s, &conv, &rec);
    GFCC_CHECK(rec.n > 0, GFCC_E_STATE, "training solves produced no restart pairs (lower pair_restart)");
    // keep pairs whose right-hand side converged (X* = its solution) and, with xstar_ratio > 0,
    // pairs of a right-hand side stopped at data_max_iter whose residual is at least
    // xstar_ratio times that of its last iterate (X* = the last iterate)
    const double ratio = mo->struct_size >= offsetof(gfcc_mlp_opts, xstar_ratio) + sizeof(double)
                             ? mo->xstar_ratio : 0.0;
    GFCC_CHECK(ratio >= 0.0 && std::isfinite(ratio), GFCC_E_ARG, "bad xstar_ratio");
    std::vector<int> keep;
    for (int64_t k = 0; k < rec.n; ++k) {
      const size_t r = size_t(rec.rhs[size_t(k)]);
      const double fin = r < rec.final_nrm.size() ? rec.final_nrm[r] : 0.0;
      if (inf[r].status == 0 || (ratio > 0.0 && inf[r].status == 1 && fin > 0.0 && rec.nrm[size_t(k)] >= ratio * fin))
        keep.push_back(int(k));
    }
    GFCC_CHECK(!keep.empty(), GFCC_E_STATE,
               "no training pair: no right-hand side converged and none qualified under xstar_ratio");
    const int64_t npairs = rec.n;
    bE.ensure(size_t(npairs) * 2 * Dp * 8, s);
    DBuf drhs, dom, dnr;
    std::vector<int> rh(rec.rhs.begin(), rec.rhs.end());
    drhs.ensure(rh.size() * sizeof(int), s);
    GFCC_HIP(hipMemcpyAsync(drhs.p, rh.data(), rh.size() * sizeof(int), hipMemcpyHostToDevice, s));
    mlp_pair_errors(bE.as<double>(), rec.X, rec.xstar, drhs.as<int>(), npairs, Dp, s);
    // compact the kept pairs to the front (in place, order preserved)
    std::vector<double> om, nr;
    for (size_t i = 0; i < keep.size(); ++i) {
      const int k = keep[i];
      if (int64_t(i) != k) {
        GFCC_HIP(hipMemcpyAsync(bR.as<double>() + i * 2 * Dp, bR.as<double>() + k * 2 * Dp, size_t(2 * Dp) * 8,
                                hipMemcpyDeviceToDevice, s));
        GFCC_HIP(hipMemcpyAsync(bE.as<double>() + i * 2 * Dp, bE.as<double>() + k * 2 * Dp, size_t(2 * Dp) * 8,
                                hipMemcpyDeviceToDevice, s));
      }
      om.push_back(rec.omega[size_t(k)]);
      nr.push_back(rec.nrm[size_t(k)]);
    }
    dom.ensure(om.size() * 8, s);
    dnr.ensure(nr.size() * 8, s);
    GFCC_HIP(hipMemcpyAsync(dom.p, om.data(), om.size() * 8, hipMemcpyHostToDevice, s));
    GFCC_HIP(hipMemcpyAsync(dnr.p, nr.data(), nr.size() * 8, hipMemcpyHostToDevice, s));
    GFCC_HIP(hipStreamSynchronize(s));
    const auto t1 = std::chrono::steady_clock::now();
    // 2. training
    MlpPairs pr;
    pr.R = bR.as<double>();
    pr.E = bE.as<double>();
    pr.omega = dom.as<double>();
    pr.nrm = dnr.as<double>();
    pr.n = int64_t(keep.size());
    gfcc_mlp_report r{};
    mlp_train(c, pr, mo->steps, mo->batch, mo->lr, mo->seed, eta, &r, s);
    const auto t2 = std::chrono::steady_clock::now();
    r.n_pairs = pr.n;
    r.data_seconds = std::chrono::duration<double>(t1 - t0).count();
    r.train_seconds = std::chrono::duration<double>(t2 - t1).count();
    if (rep) *rep = r;
  });
}

// ---------------------------------------------------------------- model-order reduction

gfcc_status gfcc_mor_reset(gfcc_ctx* c) {
  return guarded([&] {
    ip_sector(c, "gfcc_mor_reset");
    GFCC_CHECK(c, GFCC_E_ARG, "null context");
    mor_reset(c);
  });
}

gfcc_status gfcc_mor_extend(gfcc_ctx* c, int64_t n, const double* X, double drop_tol, int64_t* m_out,
                            void* stream) {
  return guarded([&] {
    ip_sector(c, "gfcc_mor_extend");
    GFCC_CHECK(c, GFCC_E_ARG, "null context");
    GFCC_CHECK(n >= 0, GFCC_E_ARG, "n < 0");
    GFCC_CHECK(drop_tol >= 0.0 && drop_tol < 1.0, GFCC_E_ARG, "drop_tol must be in [0, 1)");
    if (n > 0) {
      GFCC_CHECK(X, GFCC_E_ARG, "null X");
      mor_extend(c, n, X, drop_tol, as_stream(stream), nullptr, nullptr);
    }
    if (m_out) *m_out = mor_size(c);
  });
}

// orbital indices in [0, limit)
static void check_pq(int64_t limit, int64_t n, const int64_t* v, const char* what) {
  GFCC_CHECK(v, GFCC_E_ARG, std::string("null ") + what);
  for (int64_t k = 0; k < n; ++k)
    GFCC_CHECK(v[k] >= 0 && v[k] < limit, GFCC_E_ARG, std::string(what) + " out of range");
}

gfcc_status gfcc_mor_model(gfcc_ctx* c, int64_t np, const int64_t* p, int64_t nq, const int64_t* q,
                           int64_t n_omega, const double* omega, double eta, double* G, void* stream) {
  return guarded([&] {
    ip_sector(c, "gfcc_mor_model");
    GFCC_CHECK(c, GFCC_E_ARG, "null context");
    GFCC_CHECK(np >= 1 && n_omega >= 0 && (q == nullptr || nq >= 1), GFCC_E_ARG, "bad sizes");
    if (n_omega == 0) return;
    check_pq(c->o, np, p, "p (occupied: the model right-hand side is S^T e_p)");
    if (q) check_pq(c->o + c->v, nq, q, "q");
    GFCC_CHECK(omega && G, GFCC_E_ARG, "null argument");
    for (int64_t k = 0; k < n_omega; ++k) GFCC_CHECK(std::isfinite(omega[k]), GFCC_E_ARG, "non-finite omega");
    mor_model(c, np, p, q ? nq : np, q, q == nullptr, n_omega, omega, eta, G, as_stream(stream));
  });
}

gfcc_status gfcc_mor_export(gfcc_ctx* c, int32_t which, double* dst, int64_t* m_out, void* stream) {
  return guarded([&] {
    ip_sector(c, "gfcc_mor_export");
    GFCC_CHECK(c, GFCC_E_ARG, "null context");
    GFCC_CHECK(which == 0 || which == 1, GFCC_E_ARG, "which must be 0 (Hhat) or 1 (basis)");
    if (m_out) *m_out = mor_size(c);
    if (dst) {
      hipStream_t s = as_stream(stream);
      mor_export(c, which, dst, s);
      GFCC_HIP(hipStreamSynchronize(s));
    }
  });
}

gfcc_status gfcc_mor_greens(gfcc_ctx* c, int64_t np, const int64_t* p, int64_t n_omega, const double* omega,
                            double eta, const gfcc_mor_opts* opts, double* G, int32_t* level_of,
                            gfcc_mor_report* report, void* stream) {
  bool all_conv = true;
  gfcc_status st = guarded([&] {
    ip_sector(c, "gfcc_mor_greens");
    GFCC_CHECK(c, GFCC_E_ARG, "null context");
    GFCC_CHECK(opts && opts->struct_size >= sizeof(gfcc_mor_opts), GFCC_E_ARG, "bad options struct");
    GFCC_CHECK(opts->solve.struct_size >= sizeof(gfcc_solve_opts), GFCC_E_ARG, "bad solve options struct");
    GFCC_CHECK(np >= 1 && n_omega >= 1, GFCC_E_ARG, "np and n_omega must be >= 1");
    check_pq(c->o, np, p, "p (occupied)");
    GFCC_CHECK(omega && G, GFCC_E_ARG, "null argument");
    GFCC_CHECK(opts->tol > 0.0 && opts->drop_tol >= 0.0 && opts->drop_tol < 1.0 && opts->max_levels >= 0,
               GFCC_E_ARG, "bad tol / drop_tol / max_levels");
    const gfcc_solve_opts& so = opts->solve;
    GFCC_CHECK(so.tol > 0.0 && so.restart >= 1 && so.max_iter >= 1, GFCC_E_ARG, "bad solve tolerance/restart/max_iter");
    GFCC_CHECK(so.precond >= GFCC_PC_NONE && so.precond <= GFCC_PC_MLP, GFCC_E_ARG, "bad preconditioner");
    GFCC_CHECK(so.precision >= GFCC_FP64 && so.precision <= GFCC_FP16_IR, GFCC_E_ARG, "bad precision");
    for (int64_t k = 0; k < n_omega; ++k) GFCC_CHECK(std::isfinite(omega[k]), GFCC_E_ARG, "non-finite omega");
    if (n_omega >= 3) {
      const double dw = (omega[n_omega - 1] - omega[0]) / double(n_omega - 1);
      GFCC_CHECK(dw > 0.0, GFCC_E_ARG, "omega must be ascending");
      for (int64_t k = 0; k < n_omega; ++k)
        GFCC_CHECK(std::fabs(omega[k] - (omega[0] + double(k) * dw)) <= 1e-9 * (std::fabs(dw) + std::fabs(omega[k])),
                   GFCC_E_ARG, "omega must be a uniform grid");
    }
    mor_greens(c, np, p, n_omega, omega, eta, opts, G, level_of, report, as_stream(stream), &all_conv);
  });
  if (st == GFCC_OK && !all_conv) return GFCC_W_NOCONV;
  return st;
}

gfcc_status gfcc_prof_enable(gfcc_ctx* c, int enable) {
  return guarded([&] {
    GFCC_CHECK(c, GFCC_E_ARG, "null context");
    prof_collect(c);
    c->prof.clear();
    c->prof_on = enable != 0;
  });
}

gfcc_status gfcc_prof_get(gfcc_ctx* c, const char* name, int64_t* count, double* ms, double* flops, double* bytes) {
  return guarded([&] {
    GFCC_CHECK(c && name, GFCC_E_ARG, "null argument");
    prof_collect(c);
    auto it = c->prof.find(name);
    gfcc_prof_entry e;
    if (it != c->prof.end()) e = it->second;
    if (count) *count = e.count;
    if (ms) *ms = e.ms;
    if (flops) *flops = e.flops;
    if (bytes) *bytes = e.bytes;
  });
}

gfcc_status gfcc_destroy(gfcc_ctx* c) {
  return guarded([&] {
    if (!c) return;
    (void)hipDeviceSynchronize();
    prof_collect(c);
    delete c;
  });
}

const char* gfcc_strerror(gfcc_status st) {
  switch (st) {
    case GFCC_OK: return "success";
    case GFCC_E_ARG: return "invalid argument";
    case GFCC_E_OOM: return "out of device memory";
    case GFCC_E_HIP: return "HIP runtime error";
    case GFCC_E_STATE: return "invalid state";
    case GFCC_W_NOCONV: return "some right-hand sides did not converge";
  }
  return "unknown status";
}

const char* gfcc_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

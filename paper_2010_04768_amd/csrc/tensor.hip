// Tensor utilities: strided permutation, a pairwise contraction engine built on
// the MFMA GEMM, and precision conversion.  Used to build the similarity-
// transformed Hamiltonian blocks once per system (the paper precomputes its
// constant intermediates before the GFCC loop; its tensor layer turns each
// contraction into GEMM-like kernels -- here: permute to K-contiguous
// operands, one MFMA GEMM, permute-accumulate the result).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "gfcc_internal.h"

namespace gfcc {

TView tview(double* p, std::initializer_list<int64_t> dims) {
  TView v;
  v.p = p;
  v.nd = int(dims.size());
  int k = 0;
  for (int64_t d : dims) v.dim[k++] = d;
  int64_t s = 1;
  for (int i = v.nd - 1; i >= 0; --i) {
    v.str[i] = s;
    s *= v.dim[i];
  }
  return v;
}

TView tview_s(double* p, std::initializer_list<int64_t> dims, std::initializer_list<int64_t> strides) {
  TView v;
  v.p = p;
  v.nd = int(dims.size());
  int k = 0;
  for (int64_t d : dims) v.dim[k++] = d;
  k = 0;
  for (int64_t s : strides) v.str[k++] = s;
  return v;
}

struct PermArgs {
  int nd;
  int64_t dim[8];
  int64_t ostr[8];
  int64_t istr[8];
  const double* in;
  double* out;
  double alpha, beta;
  int64_t total;
};

__global__ void permute_kernel(PermArgs a) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < a.total; t += stride) {
    int64_t r = t, oo = 0, io = 0;
    for (int d = a.nd - 1; d >= 0; --d) {
      const int64_t x = r % a.dim[d];
      r /= a.dim[d];
      oo += x * a.ostr[d];
      io += x * a.istr[d];
    }
    const double v = a.alpha * a.in[io];
    a.out[oo] = (a.beta == 0.0) ? v : v + a.beta * a.out[oo];
  }
}

static unsigned grid_for(int64_t n, int threads = 256) {
  int64_t b = (n + threads - 1) / threads;
  return unsigned(std::min<int64_t>(std::max<int64_t>(b, 1), 65536));
}

void permute(const TView& in, const int* perm, double alpha, const TView& out, double beta,
             hipStream_t s) {
  GFCC_CHECK(in.nd == out.nd && in.nd <= 8, GFCC_E_ARG, "permute: rank mismatch");
  PermArgs a;
  a.nd = out.nd;
  for (int d = 0; d < out.nd; ++d) {
    GFCC_CHECK(out.dim[d] == in.dim[perm[d]], GFCC_E_ARG, "permute: dimension mismatch");
    a.dim[d] = out.dim[d];
    a.ostr[d] = out.str[d];
    a.istr[d] = in.str[perm[d]];
  }
  a.in = in.p;
  a.out = out.p;
  a.alpha = alpha;
  a.beta = beta;
  a.total = out.size();
  if (a.total == 0) return;
  hipLaunchKernelGGL(permute_kernel, dim3(grid_for(a.total)), dim3(256), 0, s, a);
  GFCC_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ contraction engine

static bool is_contig(const TView& v) {
  int64_t s = 1;
  for (int i = v.nd - 1; i >= 0; --i) {
    if (v.dim[i] != 1 && v.str[i] != s) return false;
    s *= v.dim[i];
  }
  return true;
}

// If `v` (labels `vl` == rows + cols) is a row-major matrix whose column
// dims are contiguous and whose row dims advance by a uniform row stride
// ld >= #cols, return ld; otherwise -1.
static int64_t matrix_ld(const TView& v, const std::string& vl, const std::string& rows,
                         const std::string& cols) {
  if (vl != rows + cols) return -1;
  const int nr = int(rows.size());
  int64_t s = 1;
  for (int i = v.nd - 1; i >= nr; --i) {
    if (v.dim[i] != 1 && v.str[i] != s) return -1;
    s *= v.dim[i];
  }
  const int64_t ncols = s;
  if (nr == 0) return ncols;
  int64_t ld = -1;
  int64_t acc = 1;
  for (int i = nr - 1; i >= 0; --i) {
    if (v.dim[i] == 1) continue;
    if (ld < 0) {
      ld = v.str[i];
      if (ld < ncols) return -1;
      acc = ld * v.dim[i];
    } else {
      if (v.str[i] != acc) return -1;
      acc *= v.dim[i];
    }
  }
  return ld < 0 ? ncols : ld;
}

// Copy `src` (labels `sl`) into a padded row-major matrix [rows = row labels]
// [cols = col labels] with row stride `ld`; returns a view-free pointer.
static void to_matrix(const TView& src, const std::string& sl, const std::string& rows,
                      const std::string& cols, double* dst, int64_t ld, hipStream_t s) {
  std::string order = rows + cols;
  TView out;
  out.p = dst;
  out.nd = int(order.size());
  int perm[8];
  for (int d = 0; d < out.nd; ++d) {
    perm[d] = int(sl.find(order[d]));
    out.dim[d] = src.dim[perm[d]];
  }
  // strides: cols contiguous, rows with stride ld
  int64_t st = 1;
  for (int d = out.nd - 1; d >= int(rows.size()); --d) {
    out.str[d] = st;
    st *= out.dim[d];
  }
  st = ld;
  for (int d = int(rows.size()) - 1; d >= 0; --d) {
    out.str[d] = st;
    st *= out.dim[d];
  }
  permute(src, perm, 1.0, out, 0.0, s);
}

// Large products go to the 256x128 tile with direct-to-LDS loads (the FP64 ring GEMMs' tile);
// the rest to the default tile or split-K.
static void contract_gemm(const GemmArgs& g, Scratch& scr, hipStream_t s) {
  if (g.M >= 2048 && g.N >= 2048 && g.batch == 1 && !g.b_ncontig)
    gemm(Prec::F64, g, TILE_DMA2_256x128, s);
  else
    gemm_auto(Prec::F64, g, scr, 3, s);
}

void ein(const char* spec, double alpha, const TView& A, const TView& B, double beta,
         const TView& C, Scratch& scr, hipStream_t s) {
  std::string sp(spec);
  const size_t comma = sp.find(','), arrow = sp.find("->");
  GFCC_CHECK(comma != std::string::npos && arrow != std::string::npos, GFCC_E_ARG, "ein: bad spec");
  const std::string la = sp.substr(0, comma), lb = sp.substr(comma + 1, arrow - comma - 1),
                    lc = sp.substr(arrow + 2);
  GFCC_CHECK(int(la.size()) == A.nd && int(lb.size()) == B.nd && int(lc.size()) == C.nd, GFCC_E_ARG,
             std::string("ein: rank mismatch in ") + spec);
  auto dim_of = [&](char c) -> int64_t {
    size_t p;
    if ((p = la.find(c)) != std::string::npos) return A.dim[p];
    if ((p = lb.find(c)) != std::string::npos) return B.dim[p];
    return C.dim[lc.find(c)];
  };
  std::string ml, nl, kl;
  for (char c : lc) {
    const bool ina = la.find(c) != std::string::npos, inb = lb.find(c) != std::string::npos;
    GFCC_CHECK(ina != inb, GFCC_E_ARG, std::string("ein: label in C must be in exactly one input: ") + spec);
    (ina ? ml : nl) += c;
  }
  for (char c : la)
    if (lc.find(c) == std::string::npos) {
      GFCC_CHECK(lb.find(c) != std::string::npos, GFCC_E_ARG, std::string("ein: dangling label ") + spec);
      kl += c;
    }
  for (char c : lb)
    GFCC_CHECK(lc.find(c) != std::string::npos || la.find(c) != std::string::npos, GFCC_E_ARG,
               std::string("ein: dangling label ") + spec);
  for (char c : lc) GFCC_CHECK(dim_of(c) == C.dim[lc.find(c)], GFCC_E_ARG, "ein: dim mismatch");
  int64_t M = 1, N = 1, K = 1;
  for (char c : ml) M *= dim_of(c);
  for (char c : nl) N *= dim_of(c);
  for (char c : kl) K *= dim_of(c);
  if (M == 0 || N == 0) return;
  const int64_t ldk = round_up(K, 8);

  // operands as K-contiguous matrices (reuse in place when already laid out so)
  const double* pa;
  const double* pb;
  int64_t lda, ldb;
  const int64_t lda0 = matrix_ld(A, la, ml, kl), ldb0 = matrix_ld(B, lb, nl, kl);
  if (lda0 >= 0) {
    pa = A.p;
    lda = lda0;
  } else {
    double* d = scr.get(0, M * ldk, s);
    to_matrix(A, la, ml, kl, d, ldk, s);
    pa = d;
    lda = ldk;
  }
  if (ldb0 >= 0) {
    pb = B.p;
    ldb = ldb0;
  } else {
    double* d = scr.get(1, N * ldk, s);
    to_matrix(B, lb, nl, kl, d, ldk, s);
    pb = d;
    ldb = ldk;
  }
  GemmArgs g;
  g.A = pa;
  g.am = lin(lda);
  g.B = pb;
  g.bm = lin(ldb);
  g.M = M;
  g.N = N;
  g.K = K;
  const int64_t ldc0 = matrix_ld(C, lc, ml, nl);
  if (ldc0 >= 0) {
    g.C = C.p;
    g.cm = lin(ldc0);
    g.cn = lin(1);
    g.alpha = alpha;
    g.beta = beta;
    contract_gemm(g, scr, s);
    return;
  }
  double* tmp = scr.get(2, M * N, s);
  g.C = tmp;
  g.cm = lin(N);
  g.cn = lin(1);
  g.alpha = 1.0;
  g.beta = 0.0;
  contract_gemm(g, scr, s);
  // permute-accumulate tmp[ml nl] into C[lc]
  std::string tl = ml + nl;
  TView tv;
  tv.p = tmp;
  tv.nd = int(tl.size());
  int64_t st = 1;
  for (int d = tv.nd - 1; d >= 0; --d) {
    tv.dim[d] = dim_of(tl[d]);
    tv.str[d] = st;
    st *= tv.dim[d];
  }
  int perm[8];
  for (int d = 0; d < C.nd; ++d) perm[d] = int(tl.find(lc[d]));
  permute(tv, perm, alpha, C, beta, s);
}

// ------------------------------------------------------------------ conversions

__global__ void convert_kernel(const double* __restrict__ src, void* __restrict__ dst, int prec,
                               int64_t n, double scale) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n; t += stride) {
    const double v = src[t] * scale;
    if (prec == int(Prec::F32))
      static_cast<float*>(dst)[t] = float(v);
    else if (prec == int(Prec::BF16))
      static_cast<__bf16*>(dst)[t] = __bf16(float(v));
    else if (prec == int(Prec::F16))
      static_cast<_Float16*>(dst)[t] = _Float16(float(v));
    else
      static_cast<double*>(dst)[t] = v;
  }
}

void convert_f64(const double* src, void* dst, Prec p, int64_t n, double scale, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(convert_kernel, dim3(grid_for(n)), dim3(256), 0, s, src, dst, int(p), n, scale);
  GFCC_HIP(hipGetLastError());
}

__global__ void amax_kernel(const double* __restrict__ src, int64_t n, double* __restrict__ part) {
  __shared__ double red[256];
  double m = 0.0;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n; t += stride)
    m = fmax(m, fabs(src[t]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

double amax_host(const double* src, int64_t n, hipStream_t s, Scratch& scr) {
  if (n <= 0) return 0.0;
  const unsigned nb = std::min<unsigned>(grid_for(n), 1024);
  double* part = scr.get(3, nb, s);
  hipLaunchKernelGGL(amax_kernel, dim3(nb), dim3(256), 0, s, src, n, part);
  GFCC_HIP(hipGetLastError());
  std::vector<double> h(nb);
  GFCC_HIP(hipMemcpyAsync(h.data(), part, nb * sizeof(double), hipMemcpyDeviceToHost, s));
  GFCC_HIP(hipStreamSynchronize(s));
  double m = 0.0;
  for (double x : h) m = std::max(m, x);
  return m;
}

}  // namespace gfcc

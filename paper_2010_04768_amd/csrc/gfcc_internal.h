// Internal declarations of the gfcc library (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/gfcc.h"

namespace gfcc {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
struct Error {
  gfcc_status st;
  std::string msg;
};

#define GFCC_HIP(expr)                                                              \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess) {                                                         \
      (void)hipGetLastError(); /* do not leave the error for the caller's next check */ \
      throw ::gfcc::Error{GFCC_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_) + \
                                          " (" + __FILE__ + ":" + std::to_string(__LINE__) + ")"}; \
    }                                                                               \
  } while (0)

#define GFCC_CHECK(cond, status, msg)                                      \
  do {                                                                     \
    if (!(cond)) throw ::gfcc::Error{status, std::string(msg)};            \
  } while (0)

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// ---------------------------------------------------------------- device memory
// Incremented whenever a library buffer is (re)allocated; captured HIP graphs
// hold raw addresses and are discarded when it changes.
inline uint64_t& alloc_generation() {
  static thread_local uint64_t g = 0;
  return g;
}

struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; bytes = o.bytes; o.p = nullptr; o.bytes = 0; }
    return *this;
  }
  ~DBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  // (re)allocate at least n bytes, zero-filled on the given stream when grown
  void ensure(size_t n, hipStream_t s) {
    if (n <= bytes && p) return;
    if (p) GFCC_HIP(hipStreamSynchronize(s));  // old buffer may still be in use on s
    release();
    if (n == 0) n = 256;
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) {
      p = nullptr;
      throw Error{GFCC_E_OOM, "hipMalloc of " + std::to_string(n) + " bytes failed"};
    }
    bytes = n;
    ++alloc_generation();
    GFCC_HIP(hipMemsetAsync(p, 0, n, s));
  }
  template <typename T> T* as() const { return static_cast<T*>(p); }
};

// ---------------------------------------------------------------- GEMM
// C(i, j) = alpha * sum_k A(i, k) B(j, k) + beta * C(i, j)
// Operand rows are K-contiguous; a row's element offset is given by a two-level
// map  off(r) = (r / div) * hi + (r % div) * lo  (div >= 1).
struct RowMap {
  int64_t div, hi, lo;
};
inline RowMap lin(int64_t ld) { return RowMap{int64_t(1) << 40, 0, ld}; }
inline RowMap two(int64_t div, int64_t hi, int64_t lo) { return RowMap{div, hi, lo}; }

enum class Prec : int { F64 = 0, F32 = 1, BF16 = 2, F16 = 3 };

struct GemmArgs {
  const void* A = nullptr;  // element type given by Prec
  RowMap am{};              // row i of A starts at am(i); K contiguous
  const void* B = nullptr;
  RowMap bm{};              // b_ncontig == 0: row j of B at bm(j), K contiguous
                            // b_ncontig == 1: K-row k of B at bm(k), N contiguous
  int b_ncontig = 0;
  double* C = nullptr;
  RowMap cm{}, cn{};
  RowMap az{int64_t(1) << 40, 0, 0}, bz{int64_t(1) << 40, 0, 0}, cz{int64_t(1) << 40, 0, 0};  // batch offsets
  int64_t M = 0, N = 0, K = 0;
  int batch = 1;
  double alpha = 1.0, beta = 0.0;
  // when set, the epilogue multiplies alpha by *alpha_dev (a device scalar: the inverse of an
  // operand scale computed on the GPU, so that no host round trip sits between the two)
  const double* alpha_dev = nullptr;
  // split-K: when > 0, grid.z indexes K slices of this length; slice z reads
  // columns [z*k_split, min(K, (z+1)*k_split)) and writes its partial sum to
  // C + cz(z) with alpha = 1, beta = 0 (batch must then equal the slice count)
  int64_t k_split = 0;
};

// Several independent GEMMs (same precision and tile) in one launch.
constexpr int MAX_GEMM_GROUPS = 4;
struct GemmGroup {
  GemmArgs g[MAX_GEMM_GROUPS];
  int64_t start[MAX_GEMM_GROUPS + 1];  // first block of each group (multiples of 8)
  int ng = 0;
};

// Tile configurations; the autotuner picks one per (shape, precision).
enum TileCfg : int {
  TILE_128x128 = 0, TILE_64x64 = 1, TILE_128x64 = 2, TILE_64x128 = 3,
  // double-buffered LDS, one barrier per K-step (K-contiguous B only)
  TILE_DB_128x128 = 4, TILE_DB_256x128 = 5, TILE_DB_128x256 = 6, TILE_DB_256x256 = 7,
  // double-buffered with 32x32x16 BF16 MFMA blocks (other types: the 16x16 kernel of the same tile)
  TILE_DB32_256x256 = 8, TILE_DB32_256x128 = 9, TILE_DB32_128x128 = 10,
  // 256x256 with 16 waves of 64x64 (BF16; other types: the 8-wave kernel of the same tile)
  TILE_DB32_256x256_W16 = 11, TILE_DB_256x256_W16 = 12,
  // 16-bit types: 256x256 tiles with loads straight into LDS stages of K = 32: 3 or 4 stages and
  // 16 waves of 64x64, 3 stages and 8 waves of 128x64 or 64x128; or 2 stages of K = 64 and 16
  // waves (others: the 16-wave tile above)
  TILE_DMA3_256x256 = 13, TILE_DMA4_256x256 = 14, TILE_DMA3_256x256_W8 = 15, TILE_DMA3_256x256_W8T = 16,
  TILE_DMA2K64_256x256 = 17,
  // FP64 and FP32: 256x128 tiles, 8 waves of 64x64, loads straight into 3 or 2 LDS stages of
  // 128-byte rows (K = 16 doubles or 32 floats; other types: the double-buffered 256x128 tile)
  TILE_DMA3_256x128 = 18, TILE_DMA2_256x128 = 19,
  // FP64: 128x256, 8 waves of 64x64, two LDS stages of K = 16 (other types: the double-buffered 128x256)
  TILE_DMA2_128x256 = 20,
  N_TILE_CFG = 21
};
const char* tile_name(int cfg);

void gemm(Prec p, const GemmArgs& a, int cfg, hipStream_t s);
// ng <= MAX_GEMM_GROUPS GEMMs (batch 1, no split-K, K-contiguous B) in one grouped launch
void gemm_grouped(Prec p, const GemmArgs* a, int ng, int cfg, hipStream_t s);
// GEMM whose tile grid is too small to fill the GPU: split K over `slices`,
// reduce the partials (deterministic order) into C with alpha/beta.
void gemm_splitk(Prec p, const GemmArgs& a, int slices, double* part, hipStream_t s);
int splitk_slices(int64_t M, int64_t N, int64_t K);
// heuristic choice when no tuned entry exists
int gemm_default_cfg(int64_t M, int64_t N, int64_t K);
// precision-aware choice for large K-contiguous products (double-buffered tiles)
int gemm_big_cfg(Prec p, int64_t M, int64_t N, int64_t K);

// reduced-precision form of a solver precision: index of the context's copy set and element type
inline int lowp_index(gfcc_precision p) { return p == GFCC_BF16_IR ? 1 : (p == GFCC_FP16_IR ? 2 : 0); }
inline Prec inner_prec(gfcc_precision p) {
  return p == GFCC_FP64 ? Prec::F64 : (p == GFCC_FP32_IR ? Prec::F32 : (p == GFCC_BF16_IR ? Prec::BF16 : Prec::F16));
}

// ---------------------------------------------------------------- tensors
struct TView {
  double* p = nullptr;
  int nd = 0;
  int64_t dim[8] = {0};
  int64_t str[8] = {0};
  int64_t size() const {
    int64_t s = 1;
    for (int i = 0; i < nd; ++i) s *= dim[i];
    return s;
  }
};
TView tview(double* p, std::initializer_list<int64_t> dims);                 // contiguous
TView tview_s(double* p, std::initializer_list<int64_t> dims, std::initializer_list<int64_t> strides);

// out = alpha * permute(in) + beta * out ; `in` and `out` have the same number
// of dims; out dim d takes in dim perm[d].
void permute(const TView& in, const int* perm, double alpha, const TView& out, double beta,
             hipStream_t s);

// Scratch arena reused by the contraction engine.
struct Scratch {
  DBuf b[8];
  double* get(int slot, int64_t n, hipStream_t s) {
    b[slot].ensure(size_t(n) * sizeof(double), s);
    return b[slot].as<double>();
  }
};

// gemm, or gemm_splitk with partials in scr slot `scr_slot` when the tile grid is small
void gemm_auto(Prec p, const GemmArgs& a, Scratch& scr, int scr_slot, hipStream_t s);

// Pairwise contraction  C[c] = alpha * sum A[a] B[b] + beta * C[c]  in FP64 on
// MFMA.  `spec` is "ab..,cd..->ef.." with single-letter labels; every label is
// in exactly two of the three operands.
void ein(const char* spec, double alpha, const TView& A, const TView& B, double beta,
         const TView& C, Scratch& scr, hipStream_t s);

// ---------------------------------------------------------------- conversions
void convert_f64(const double* src, void* dst, Prec p, int64_t n, double scale, hipStream_t s);
double amax_host(const double* src, int64_t n, hipStream_t s, Scratch& scr);

}  // namespace gfcc

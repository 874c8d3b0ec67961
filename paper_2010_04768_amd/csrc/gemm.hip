// MFMA GEMM for gfx950:  C(i, j) = alpha * sum_k A(i, k) B(j, k) + beta * C(i, j).
//
// Both operands are K-contiguous ("NT" form); the row of each operand and the
// row/column of C go through a two-level map so that the sigma product's index
// permutations (the (i,j,a) <- (m,e) ring contractions) are absorbed in the
// operand fetch and in the epilogue instead of extra passes over HBM.
//
// Element types: FP64 (v_mfma_f64_16x16x4f64, FP64 accumulation), FP32
// (v_mfma_f32_16x16x4f32), BF16 and FP16 (v_mfma_f32_16x16x32_{bf16,f16} and the
// 32x32x16 forms, gfx950), the last three accumulating in FP32.  C is always FP64.
//
// Tiling: a workgroup of 4 waves (2 x 2) computes a BM x BN tile; each wave a
// (BM/2) x (BN/2) sub-tile as (BM/32) x (BN/32) MFMA 16x16 blocks.  K advances
// in BK-element steps staged through LDS (rows padded by 16 bytes to spread
// banks) with the next step prefetched into registers while MFMAs run.  The
// workgroup -> tile map keeps consecutive tiles on one XCD (workgroups are
// dealt round-robin over the 8 XCDs) and walks tile-rows in groups so that
// concurrently running tiles share operand panels in that XCD's L2.
#include <algorithm>
#include <type_traits>

#include "gfcc_internal.h"

namespace gfcc {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
// Every shape below describes its lane layout to the double-buffered kernel:
// a 16x16 (or 32x32) block of C per instruction (BLK), K per instruction (KS),
// the operand row and first K element a lane supplies (frow, fk) and where
// accumulator r of a lane lands in the C block (orow, ocol).
template <> struct Mfma<double> {
  using acc_t = v4d;
  using frag_t = double;
  static constexpr int KS = 4;       // K per instruction
  static constexpr int BLK = 16, NACC = 4;
  static constexpr bool ROW_INTERLEAVED = true;  // D[(l/16) + 4r][l%16]
  __device__ static inline acc_t mma(frag_t a, frag_t b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int frow(int l) { return l & 15; }
  __device__ static inline int fk(int l) { return l >> 4; }
  __device__ static inline int orow(int l, int r) { return (l >> 4) + 4 * r; }
  __device__ static inline int ocol(int l) { return l & 15; }
};
template <> struct Mfma<float> {
  using acc_t = v4f;
  using frag_t = float;
  static constexpr int KS = 4;
  static constexpr int BLK = 16, NACC = 4;
  static constexpr bool ROW_INTERLEAVED = false;  // D[4(l/16) + r][l%16]
  __device__ static inline acc_t mma(frag_t a, frag_t b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int frow(int l) { return l & 15; }
  __device__ static inline int fk(int l) { return l >> 4; }
  __device__ static inline int orow(int l, int r) { return 4 * (l >> 4) + r; }
  __device__ static inline int ocol(int l) { return l & 15; }
};
template <> struct Mfma<__bf16> {
  using acc_t = v4f;
  using frag_t = v8bf;
  static constexpr int KS = 32;
  static constexpr int BLK = 16, NACC = 4;
  static constexpr bool ROW_INTERLEAVED = false;
  __device__ static inline acc_t mma(frag_t a, frag_t b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  __device__ static inline int frow(int l) { return l & 15; }
  __device__ static inline int fk(int l) { return (l >> 4) * 8; }
  __device__ static inline int orow(int l, int r) { return 4 * (l >> 4) + r; }
  __device__ static inline int ocol(int l) { return l & 15; }
};
template <> struct Mfma<_Float16> {
  using acc_t = v4f;
  using frag_t = v8h;
  static constexpr int KS = 32;
  static constexpr int BLK = 16, NACC = 4;
  static constexpr bool ROW_INTERLEAVED = false;
  __device__ static inline acc_t mma(frag_t a, frag_t b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
  __device__ static inline int frow(int l) { return l & 15; }
  __device__ static inline int fk(int l) { return (l >> 4) * 8; }
  __device__ static inline int orow(int l, int r) { return 4 * (l >> 4) + r; }
  __device__ static inline int ocol(int l) { return l & 15; }
};
// 32x32x16 BF16: half the instructions and fragment loads per flop of the 16x16x32 form
struct Mfma32Bf16 {
  using acc_t = v16f;
  using frag_t = v8bf;
  static constexpr int KS = 16;
  static constexpr int BLK = 32, NACC = 16;
  __device__ static inline acc_t mma(frag_t a, frag_t b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
  __device__ static inline int frow(int l) { return l & 31; }
  __device__ static inline int fk(int l) { return (l >> 5) * 8; }
  __device__ static inline int orow(int l, int r) { return 8 * (r >> 2) + 4 * (l >> 5) + (r & 3); }
  __device__ static inline int ocol(int l) { return l & 31; }
};
// the same shape in FP16 (same lane layout)
struct Mfma32F16 {
  using acc_t = v16f;
  using frag_t = v8h;
  static constexpr int KS = 16;
  static constexpr int BLK = 32, NACC = 16;
  __device__ static inline acc_t mma(frag_t a, frag_t b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
  __device__ static inline int frow(int l) { return l & 31; }
  __device__ static inline int fk(int l) { return (l >> 5) * 8; }
  __device__ static inline int orow(int l, int r) { return 8 * (r >> 2) + 4 * (l >> 5) + (r & 3); }
  __device__ static inline int ocol(int l) { return l & 31; }
};
// 16-bit element types take the 32x32x16 shape in the DB32 tiles
template <typename T> struct Wide { using type = Mfma<T>; static constexpr bool on = false; };
template <> struct Wide<__bf16> { using type = Mfma32Bf16; static constexpr bool on = true; };
template <> struct Wide<_Float16> { using type = Mfma32F16; static constexpr bool on = true; };

// Workgroups are dealt round-robin over the 8 XCDs (workgroup b runs on XCD
// b % 8).  Give XCD x a contiguous range of tiles: with ntiles = 8q + r, XCDs
// x < r take q + 1 tiles and the others q; a bijection on [0, ntiles).
__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t ntiles) {
  const int64_t q = ntiles >> 3, r = ntiles & 7;
  const int64_t x = bid & 7, idx = bid >> 3;
  return (x < r) ? x * (q + 1) + idx : r * (q + 1) + (x - r) * q + idx;
}

__device__ __forceinline__ int64_t rmap(const RowMap& m, int64_t r) {
  return (r / m.div) * m.hi + (r % m.div) * m.lo;
}

template <typename T, int BM, int BN, bool VEC, bool BNC>
__device__ __forceinline__ void gemm_tile(const GemmArgs& g, int64_t braw) {
  using MF = Mfma<T>;
  constexpr int EPC = 16 / int(sizeof(T));   // elements per 16-byte chunk
  constexpr int BK = 8 * EPC;                // 8 chunks per row: 16 fp64, 32 fp32, 64 bf16
  constexpr int LDK = BK + EPC;              // padded LDS row (144 bytes)
  constexpr int RPP = 256 / 8;               // rows per load pass
  constexpr int PA = BM / RPP, PB = BN / RPP;
  constexpr int WM = BM / 2, WN = BN / 2, FM = WM / 16, FN = WN / 16;
  constexpr int FE = (MF::KS == 32) ? 8 : 1;  // elements per lane per fragment

  __shared__ __attribute__((aligned(16))) T As[BM * LDK];
  __shared__ __attribute__((aligned(16))) T Bs[BN * LDK];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm0 = (wave >> 1) * WM;
  const int wn0 = (wave & 1) * WN;

  // ---- workgroup -> tile (XCD-aware, grouped)
  const int64_t tiles_m = (g.M + BM - 1) / BM;
  const int64_t tiles_n = (g.N + BN - 1) / BN;
  const int64_t ntiles = tiles_m * tiles_n;
  int64_t bid = braw;
  bid = xcd_remap(bid, ntiles);
  constexpr int64_t GROUP = 8;
  const int64_t per_group = GROUP * tiles_n;
  const int64_t grp = bid / per_group;
  const int64_t first_m = grp * GROUP;
  const int64_t gsz = (tiles_m - first_m) < GROUP ? (tiles_m - first_m) : GROUP;
  const int64_t in_grp = bid - grp * per_group;
  const int64_t tm = first_m + in_grp % gsz;
  const int64_t tn = in_grp / gsz;
  const int64_t i0 = tm * BM, j0 = tn * BN;

  const int z = blockIdx.z;
  const int64_t kbase = g.k_split > 0 ? z * g.k_split : 0;
  const int64_t Kz = g.k_split > 0 ? ((g.K - kbase) < g.k_split ? (g.K - kbase) : g.k_split) : g.K;
  const T* A = static_cast<const T*>(g.A) + (g.k_split > 0 ? kbase : rmap(g.az, z));
  const T* B = static_cast<const T*>(g.B) + (g.k_split > 0 ? (BNC ? 0 : kbase) : rmap(g.bz, z));
  const int64_t bk0 = (g.k_split > 0 && BNC) ? kbase : 0;  // K offset of B rows when N-contiguous

  // ---- per-thread fetch rows (fixed across the K loop)
  const int lrow = tid >> 3;        // 0..31
  const int lchunk = tid & 7;       // chunk within the row
  int64_t aoff[PA], boff[PB];
#pragma unroll
  for (int p = 0; p < PA; ++p) {
    int64_t i = i0 + lrow + p * RPP;
    aoff[p] = (i < g.M) ? rmap(g.am, i) : -1;
  }
#pragma unroll
  for (int p = 0; p < PB; ++p) {
    int64_t j = j0 + lrow + p * RPP;
    boff[p] = (!BNC && j < g.N) ? rmap(g.bm, j) : -1;
  }
  // N-contiguous B: thread loads EPC consecutive j of one K-row
  constexpr int NCH = BN / EPC;            // chunks per K-row
  constexpr int KPP = 256 / NCH;           // K-rows per pass
  constexpr int PBN = BNC ? (BK + KPP - 1) / KPP : 1;
  const int nk_row = tid / NCH, nj_ch = tid % NCH;

  u4 ra[PA], rb[BNC ? PBN : PB];
  auto fetch = [&](const T* base, int64_t off, int64_t k) -> u4 {
    u4 v = {0u, 0u, 0u, 0u};
    if (off < 0) return v;
    if (VEC && k + EPC <= Kz) {
      v = *reinterpret_cast<const u4*>(base + off + k);
    } else {
      T tmp[EPC];
#pragma unroll
      for (int e = 0; e < EPC; ++e) tmp[e] = (k + e < Kz) ? base[off + k + e] : T(0);
      v = *reinterpret_cast<const u4*>(tmp);
    }
    return v;
  };
  auto load_tiles = [&](int64_t k0) {
    const int64_t k = k0 + lchunk * EPC;
#pragma unroll
    for (int p = 0; p < PA; ++p) ra[p] = fetch(A, aoff[p], k);
    if constexpr (!BNC) {
#pragma unroll
      for (int p = 0; p < PB; ++p) rb[p] = fetch(B, boff[p], k);
    } else {
#pragma unroll
      for (int p = 0; p < PBN; ++p) {
        const int kr = nk_row + p * KPP;
        const int64_t kk = k0 + kr;
        const int64_t j = j0 + nj_ch * EPC;
        u4 v = {0u, 0u, 0u, 0u};
        if (kr < BK && kk < Kz && j < g.N) {
          const T* row = B + rmap(g.bm, bk0 + kk);
          if (VEC && j + EPC <= g.N) {
            v = *reinterpret_cast<const u4*>(row + j);
          } else {
            T tmp[EPC];
#pragma unroll
            for (int e = 0; e < EPC; ++e) tmp[e] = (j + e < g.N) ? row[j + e] : T(0);
            v = *reinterpret_cast<const u4*>(tmp);
          }
        }
        rb[p] = v;
      }
    }
  };
  auto store_tiles = [&]() {
#pragma unroll
    for (int p = 0; p < PA; ++p)
      *reinterpret_cast<u4*>(&As[(lrow + p * RPP) * LDK + lchunk * EPC]) = ra[p];
    if constexpr (!BNC) {
#pragma unroll
      for (int p = 0; p < PB; ++p)
        *reinterpret_cast<u4*>(&Bs[(lrow + p * RPP) * LDK + lchunk * EPC]) = rb[p];
    } else {
#pragma unroll
      for (int p = 0; p < PBN; ++p) {
        const int kr = nk_row + p * KPP;
        if (kr < BK) {
          const T* v = reinterpret_cast<const T*>(&rb[p]);
#pragma unroll
          for (int e = 0; e < EPC; ++e) Bs[(nj_ch * EPC + e) * LDK + kr] = v[e];
        }
      }
    }
  };

  typename MF::acc_t acc[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) acc[a][b] = typename MF::acc_t{0, 0, 0, 0};

  const int nk = int((Kz + BK - 1) / BK);
  load_tiles(0);
  const int fr = lane & 15;          // fragment row within a 16-block
  const int fk = (lane >> 4) * FE;   // fragment K offset
  for (int kt = 0; kt < nk; ++kt) {
    __syncthreads();
    store_tiles();
    __syncthreads();
    if (kt + 1 < nk) load_tiles(int64_t(kt + 1) * BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += MF::KS) {
      typename MF::frag_t af[FM], bf[FN];
#pragma unroll
      for (int a = 0; a < FM; ++a)
        af[a] = *reinterpret_cast<const typename MF::frag_t*>(&As[(wm0 + a * 16 + fr) * LDK + ks + fk]);
#pragma unroll
      for (int b = 0; b < FN; ++b)
        bf[b] = *reinterpret_cast<const typename MF::frag_t*>(&Bs[(wn0 + b * 16 + fr) * LDK + ks + fk]);
#pragma unroll
      for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) acc[a][b] = MF::mma(af[a], bf[b], acc[a][b]);
    }
  }

  // ---- epilogue
  double* C = g.C + rmap(g.cz, z);
  const double al = g.alpha_dev ? g.alpha * (*g.alpha_dev) : g.alpha;
  const int jl = lane & 15;
  const int ih = lane >> 4;
#pragma unroll
  for (int b = 0; b < FN; ++b) {
    const int64_t j = j0 + wn0 + b * 16 + jl;
    if (j >= g.N) continue;
    const int64_t cj = rmap(g.cn, j);
#pragma unroll
    for (int a = 0; a < FM; ++a) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ii = MF::ROW_INTERLEAVED ? (ih + 4 * r) : (4 * ih + r);
        const int64_t i = i0 + wm0 + a * 16 + ii;
        if (i >= g.M) continue;
        double* p = C + rmap(g.cm, i) + cj;
        const double v = al * double(acc[a][b][r]);
        *p = (g.beta == 0.0) ? v : v + g.beta * (*p);
      }
    }
  }
}

template <typename T, int BM, int BN, bool VEC, bool BNC>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g) {
  gemm_tile<T, BM, BN, VEC, BNC>(g, blockIdx.x);
}

// Double-buffered variant for the large ring GEMMs (both operands K-contiguous):
// NW = WGM x WGN waves, each computing a (BM/WGM) x (BN/WGN) sub-tile; two LDS
// stages so that one barrier per K-step separates "store next" from "read
// current"; global loads for step k+1 are issued before the MFMAs of step k.
template <typename T, typename MF, int BM, int BN, int WGM, int WGN, int KM, bool VEC>
__device__ __forceinline__ void gemm_db_tile(const GemmArgs& g, int64_t braw) {
  constexpr int NT = 64 * WGM * WGN;
  constexpr int EPC = 16 / int(sizeof(T));
  constexpr int CPR = 8 * KM;  // 16-byte chunks per K-row of a stage
  constexpr int BK = CPR * EPC;
  constexpr int LDK = BK + EPC;
  constexpr int RPP = NT / CPR;
  constexpr int PA = BM / RPP, PB = BN / RPP;
  constexpr int WM = BM / WGM, WN = BN / WGN, FM = WM / MF::BLK, FN = WN / MF::BLK;
  static_assert(PA >= 1 && PB >= 1 && BM % RPP == 0 && BN % RPP == 0, "tile/thread mismatch");
  static_assert(FM >= 1 && FN >= 1 && WM % MF::BLK == 0 && WN % MF::BLK == 0, "wave tile/MFMA mismatch");

  __shared__ __attribute__((aligned(16))) T As[2][BM * LDK];
  __shared__ __attribute__((aligned(16))) T Bs[2][BN * LDK];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm0 = (wave / WGN) * WM;
  const int wn0 = (wave % WGN) * WN;

  const int64_t tiles_m = (g.M + BM - 1) / BM;
  const int64_t tiles_n = (g.N + BN - 1) / BN;
  const int64_t ntiles = tiles_m * tiles_n;
  int64_t bid = braw;
  bid = xcd_remap(bid, ntiles);
  constexpr int64_t GROUP = 4;
  const int64_t per_group = GROUP * tiles_n;
  const int64_t grp = bid / per_group;
  const int64_t first_m = grp * GROUP;
  const int64_t gsz = (tiles_m - first_m) < GROUP ? (tiles_m - first_m) : GROUP;
  const int64_t in_grp = bid - grp * per_group;
  const int64_t tm = first_m + in_grp % gsz;
  const int64_t tn = in_grp / gsz;
  const int64_t i0 = tm * BM, j0 = tn * BN;

  const int z = blockIdx.z;
  const int64_t kbase = g.k_split > 0 ? z * g.k_split : 0;
  const int64_t Kz = g.k_split > 0 ? ((g.K - kbase) < g.k_split ? (g.K - kbase) : g.k_split) : g.K;
  const T* A = static_cast<const T*>(g.A) + (g.k_split > 0 ? kbase : rmap(g.az, z));
  const T* B = static_cast<const T*>(g.B) + (g.k_split > 0 ? kbase : rmap(g.bz, z));

  const int lrow = tid / CPR;
  const int lchunk = tid % CPR;
  int64_t aoff[PA], boff[PB];
#pragma unroll
  for (int p = 0; p < PA; ++p) {
    const int64_t i = i0 + lrow + p * RPP;
    aoff[p] = (i < g.M) ? rmap(g.am, i) : -1;
  }
#pragma unroll
  for (int p = 0; p < PB; ++p) {
    const int64_t j = j0 + lrow + p * RPP;
    boff[p] = (j < g.N) ? rmap(g.bm, j) : -1;
  }
  u4 ra[PA], rb[PB];
  auto fetch = [&](const T* base, int64_t off, int64_t k) -> u4 {
    u4 v = {0u, 0u, 0u, 0u};
    if (off < 0) return v;
    if (VEC && k + EPC <= Kz) {
      v = *reinterpret_cast<const u4*>(base + off + k);
    } else {
      T tmp[EPC];
#pragma unroll
      for (int e = 0; e < EPC; ++e) tmp[e] = (k + e < Kz) ? base[off + k + e] : T(0);
      v = *reinterpret_cast<const u4*>(tmp);
    }
    return v;
  };
  auto load_tiles = [&](int64_t k0) {
    const int64_t k = k0 + lchunk * EPC;
#pragma unroll
    for (int p = 0; p < PA; ++p) ra[p] = fetch(A, aoff[p], k);
#pragma unroll
    for (int p = 0; p < PB; ++p) rb[p] = fetch(B, boff[p], k);
  };
  auto store_tiles = [&](int buf) {
#pragma unroll
    for (int p = 0; p < PA; ++p)
      *reinterpret_cast<u4*>(&As[buf][(lrow + p * RPP) * LDK + lchunk * EPC]) = ra[p];
#pragma unroll
    for (int p = 0; p < PB; ++p)
      *reinterpret_cast<u4*>(&Bs[buf][(lrow + p * RPP) * LDK + lchunk * EPC]) = rb[p];
  };

  typename MF::acc_t acc[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) acc[a][b] = typename MF::acc_t{};

  const int nk = int((Kz + BK - 1) / BK);
  const int fr = MF::frow(lane);
  const int fk = MF::fk(lane);
  load_tiles(0);
  store_tiles(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) load_tiles(int64_t(kt + 1) * BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += MF::KS) {
      typename MF::frag_t af[FM], bf[FN];
#pragma unroll
      for (int a = 0; a < FM; ++a)
        af[a] = *reinterpret_cast<const typename MF::frag_t*>(&As[cur][(wm0 + a * MF::BLK + fr) * LDK + ks + fk]);
#pragma unroll
      for (int b = 0; b < FN; ++b)
        bf[b] = *reinterpret_cast<const typename MF::frag_t*>(&Bs[cur][(wn0 + b * MF::BLK + fr) * LDK + ks + fk]);
#pragma unroll
      for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) acc[a][b] = MF::mma(af[a], bf[b], acc[a][b]);
    }
    if (kt + 1 < nk) store_tiles(cur ^ 1);
    __syncthreads();
  }

  double* C = g.C + rmap(g.cz, z);
  const double al = g.alpha_dev ? g.alpha * (*g.alpha_dev) : g.alpha;
  const int jl = MF::ocol(lane);
#pragma unroll
  for (int b = 0; b < FN; ++b) {
    const int64_t j = j0 + wn0 + b * MF::BLK + jl;
    if (j >= g.N) continue;
    const int64_t cj = rmap(g.cn, j);
#pragma unroll
    for (int a = 0; a < FM; ++a) {
#pragma unroll
      for (int r = 0; r < MF::NACC; ++r) {
        const int64_t i = i0 + wm0 + a * MF::BLK + MF::orow(lane, r);
        if (i >= g.M) continue;
        double* p = C + rmap(g.cm, i) + cj;
        const double v = al * double(acc[a][b][r]);
        *p = (g.beta == 0.0) ? v : v + g.beta * (*p);
      }
    }
  }
}

template <typename T, typename MF, int BM, int BN, int WGM, int WGN, int KM, bool VEC>
__global__ __launch_bounds__(64 * WGM * WGN) void gemm_db_kernel(GemmArgs g) {
  gemm_db_tile<T, MF, BM, BN, WGM, WGN, KM, VEC>(g, blockIdx.x);
}

// ---------------------------------------------------------------- direct-to-LDS pipeline
// 16-bit operands, 256 x 256 tile, 16 waves of 64 x 64 (32x32x16 MFMA blocks), K in steps of
// 32 through NS LDS stages.  Each step is one global_load_lds_dwordx4 per wave and operand:
// lane l of wave w moves one 16-byte chunk straight into LDS at byte (64 w + l) * 16 of the
// stage, i.e. row r = (64 w + l) / 4, slot l % 4 of a 64-byte row; the chunk it fetches is
// k-chunk slot ^ ((r / 4) % 4) of that row, so the fragment reads (16 lanes = 16 rows of one
// k-chunk) meet 16 different bank groups.  Loads run NS - 1 steps ahead with no register
// staging; a wave waits only for its own loads of the step it is about to read
// (s_waitcnt vmcnt) and a barrier then publishes every wave's part of the stage.  The loads
// are issued from inline assembly (they write no register), so the compiler adds no waits of
// its own for them: every wait on them is the explicit one below.  Operand rows are clamped
// into range (their products land outside C and are dropped); a K remainder below 32 is
// staged through registers with zero fill.  K is summed in 16-element MFMA steps in
// ascending order, as in the double-buffered kernels, so both give the same bits.
typedef __attribute__((address_space(3))) void* lds_void_ptr;

// M0 holds the wave's LDS destination (the same for every lane); lane l lands at M0 + 16 l.
// M0 is written here only; no compiler-generated code in these kernels reads it.
__device__ __forceinline__ void lds_dma16(const void* src, void* lds_dst) {
  const uint32_t m0v = __builtin_amdgcn_readfirstlane(uint32_t(uintptr_t(lds_void_ptr(lds_dst))));
  asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off" ::"v"(src), "s"(m0v) : "memory", "m0");
}
// s_waitcnt with vmcnt(n) and lgkmcnt(0) (expcnt not waited): gfx9 encoding
template <int N>
__device__ __forceinline__ void wait_vm_lgkm0() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4));
}
__device__ __forceinline__ void wg_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// Slot permutation of the 16-byte k-chunks of row r (CPR chunks per row), chosen by measurement
// (no LDS bank conflicts counted for the fragment reads): rows r and r + 16 / CPR .. of one
// k-chunk spread over the 16-byte bank groups of a 256-byte bank row.
template <int CPR>
__device__ __forceinline__ int dma_swz(int r) {
  return (r / (16 / CPR)) % CPR;
}

template <typename T, typename MF, int NS, int WGM, int WGN, int BK, int BM = 256, int BN = 256>
__device__ __forceinline__ void gemm_dma_tile(const GemmArgs& g, int64_t braw) {
  constexpr int NT = 64 * WGM * WGN;
  constexpr int WM = BM / WGM, WN = BN / WGN, FM = WM / MF::BLK, FN = WN / MF::BLK;
  constexpr int EPC = 16 / int(sizeof(T));   // elements per 16-byte chunk
  constexpr int SA = BM * BK, SB = BN * BK;  // elements per operand and stage
  constexpr int CPR = BK / EPC;              // 16-byte chunks per row
  constexpr int CPTA = BM * CPR / NT, CPTB = BN * CPR / NT;  // chunks per thread and stage
  static_assert((CPR == 4 || CPR == 8) && CPTA >= 1 && CPTB >= 1 && CPTA * NT == BM * CPR &&
                    CPTB * NT == BN * CPR, "threads must divide the stage");
  static_assert(NS * (SA + SB) * int(sizeof(T)) <= 160 * 1024, "LDS");
  static_assert(BK % MF::KS == 0 && WM % MF::BLK == 0 && WN % MF::BLK == 0, "MFMA blocks");
  static_assert(NS >= 2 && NS <= 4, "stages");
  __shared__ __attribute__((aligned(1024))) T sA0[SA];
  __shared__ __attribute__((aligned(1024))) T sB0[SB];
  __shared__ __attribute__((aligned(1024))) T sA1[SA];
  __shared__ __attribute__((aligned(1024))) T sB1[SB];
  __shared__ __attribute__((aligned(1024))) T sA2[NS > 2 ? SA : 1];
  __shared__ __attribute__((aligned(1024))) T sB2[NS > 2 ? SB : 1];
  __shared__ __attribute__((aligned(1024))) T sA3[NS > 3 ? SA : 1];
  __shared__ __attribute__((aligned(1024))) T sB3[NS > 3 ? SB : 1];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm0 = (wave / WGN) * WM;
  const int wn0 = (wave % WGN) * WN;

  const int64_t tiles_m = (g.M + BM - 1) / BM;
  const int64_t tiles_n = (g.N + BN - 1) / BN;
  const int64_t ntiles = tiles_m * tiles_n;
  int64_t bid = xcd_remap(braw, ntiles);
  constexpr int64_t GROUP = 4;
  const int64_t per_group = GROUP * tiles_n;
  const int64_t grp = bid / per_group;
  const int64_t first_m = grp * GROUP;
  const int64_t gsz = (tiles_m - first_m) < GROUP ? (tiles_m - first_m) : GROUP;
  const int64_t in_grp = bid - grp * per_group;
  const int64_t tm = first_m + in_grp % gsz;
  const int64_t tn = in_grp / gsz;
  const int64_t i0 = tm * BM, j0 = tn * BN;

  const T* A = static_cast<const T*>(g.A);
  const T* B = static_cast<const T*>(g.B);
  const int64_t Kz = g.K;
  // this thread's chunks of every stage: chunk c = p NT + tid sits at row c / CPR, slot c % CPR
  // and holds k-chunk kc[p] = slot ^ swz(row) of that row
  const T* asrc[CPTA];
  const T* bsrc[CPTB];
  // chunk p of this thread: element kc * EPC of its row (row clamped into range)
  auto chunk_kc = [&](int p) {
    const int c = p * NT + tid;
    return (c % CPR) ^ dma_swz<CPR>(c / CPR);
  };
  auto src_a = [&](int p) {
    const int r = (p * NT + tid) / CPR;
    const int64_t ia = (i0 + r < g.M) ? i0 + r : g.M - 1;
    return A + rmap(g.am, ia) + chunk_kc(p) * EPC;
  };
  auto src_b = [&](int p) {
    const int r = (p * NT + tid) / CPR;
    const int64_t jb = (j0 + r < g.N) ? j0 + r : g.N - 1;
    return B + rmap(g.bm, jb) + chunk_kc(p) * EPC;
  };
#pragma unroll
  for (int p = 0; p < CPTA; ++p) asrc[p] = src_a(p);
#pragma unroll
  for (int p = 0; p < CPTB; ++p) bsrc[p] = src_b(p);
  const int wofs = wave * 64 * EPC;  // this wave's 1 KB of a stage part, in elements

  auto stage_a = [&](auto S_) -> T* {
    constexpr int S = decltype(S_)::value;
    if constexpr (S == 0) return sA0;
    else if constexpr (S == 1) return sA1;
    else if constexpr (S == 2) return sA2;
    else return sA3;
  };
  auto stage_b = [&](auto S_) -> T* {
    constexpr int S = decltype(S_)::value;
    if constexpr (S == 0) return sB0;
    else if constexpr (S == 1) return sB1;
    else if constexpr (S == 2) return sB2;
    else return sB3;
  };
  auto issue = [&](auto S_, int64_t k0) {
#pragma unroll
    for (int p = 0; p < CPTA; ++p) lds_dma16(asrc[p] + k0, stage_a(S_) + p * NT * EPC + wofs);
#pragma unroll
    for (int p = 0; p < CPTB; ++p) lds_dma16(bsrc[p] + k0, stage_b(S_) + p * NT * EPC + wofs);
  };

  typename MF::acc_t acc[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) acc[a][b] = typename MF::acc_t{};

  // element offset within a stage of row rr, element k of the step (swizzled chunk)
  auto foff = [](int rr, int k) { return rr * BK + (((k / EPC) ^ dma_swz<CPR>(rr)) * EPC) + k % EPC; };
  const int fr = MF::frow(lane);
  const int fk = MF::fk(lane);
  auto compute = [&](const T* sa, const T* sb) {
#pragma unroll
    for (int ks = 0; ks < BK; ks += MF::KS) {
      typename MF::frag_t af[FM], bf[FN];
#pragma unroll
      for (int a = 0; a < FM; ++a)
        af[a] = *reinterpret_cast<const typename MF::frag_t*>(sa + foff(wm0 + a * MF::BLK + fr, ks + fk));
#pragma unroll
      for (int b = 0; b < FN; ++b)
        bf[b] = *reinterpret_cast<const typename MF::frag_t*>(sb + foff(wn0 + b * MF::BLK + fr, ks + fk));
#pragma unroll
      for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) acc[a][b] = MF::mma(af[a], bf[b], acc[a][b]);
    }
  };

  const int nk = int(Kz / BK);  // full steps through the pipeline
  if (nk > 0) {
    // Every step issues exactly CPTA + CPTB loads, also past the last step (then a harmless
    // re-read of step 0 into a stage nobody reads again), so the number of loads younger than
    // step kt's is always (CPTA + CPTB) (NS - 2) and each wait is one fixed count on every path.
    auto kstep = [&](int kt) { return kt < nk ? int64_t(kt) * BK : int64_t(0); };
    issue(std::integral_constant<int, 0>{}, 0);
    if constexpr (NS > 2) issue(std::integral_constant<int, 1>{}, kstep(1));
    if constexpr (NS > 3) issue(std::integral_constant<int, 2>{}, kstep(2));
    // one step: wait for step kt (stage S), publish it, refill the stage read one step ago
    // with step kt + NS - 1, compute on stage S
    auto step = [&](auto S_, int kt) {
      constexpr int S = decltype(S_)::value;
      wait_vm_lgkm0<(CPTA + CPTB) * (NS - 2)>();
      wg_barrier();
      issue(std::integral_constant<int, (S + NS - 1) % NS>{}, kstep(kt + NS - 1));
      compute(stage_a(S_), stage_b(S_));
    };
    for (int kt = 0; kt < nk; kt += NS) {
      step(std::integral_constant<int, 0>{}, kt);
      if (kt + 1 < nk) step(std::integral_constant<int, 1 % NS>{}, kt + 1);
      if constexpr (NS > 2)
        if (kt + 2 < nk) step(std::integral_constant<int, 2 % NS>{}, kt + 2);
      if constexpr (NS > 3)
        if (kt + 3 < nk) step(std::integral_constant<int, 3 % NS>{}, kt + 3);
    }
    wait_vm_lgkm0<0>();  // no load may land in LDS after the workgroup ends
  }
  if (Kz > int64_t(nk) * BK) {  // K remainder: registers, zero fill, stage 0
    u4 va[CPTA], vb[CPTB];
    auto tail_chunk = [&](const T* src, int p) {  // src: element kc * EPC of the row
      const int64_t k = int64_t(nk) * BK + chunk_kc(p) * EPC;  // absolute K index of the chunk
      T t[EPC];
#pragma unroll
      for (int e = 0; e < EPC; ++e) t[e] = (k + e < Kz) ? src[int64_t(nk) * BK + e] : T(0);
      return *reinterpret_cast<const u4*>(t);
    };
#pragma unroll
    for (int p = 0; p < CPTA; ++p) va[p] = tail_chunk(src_a(p), p);
#pragma unroll
    for (int p = 0; p < CPTB; ++p) vb[p] = tail_chunk(src_b(p), p);
    wait_vm_lgkm0<0>();
    wg_barrier();  // every wave is done with the stages
#pragma unroll
    for (int p = 0; p < CPTA; ++p) *reinterpret_cast<u4*>(sA0 + (p * NT + tid) * EPC) = va[p];
#pragma unroll
    for (int p = 0; p < CPTB; ++p) *reinterpret_cast<u4*>(sB0 + (p * NT + tid) * EPC) = vb[p];
    wait_vm_lgkm0<0>();
    wg_barrier();
    compute(sA0, sB0);
  }

  double* C = g.C;
  const double al = g.alpha_dev ? g.alpha * (*g.alpha_dev) : g.alpha;
  const int jl = MF::ocol(lane);
#pragma unroll
  for (int b = 0; b < FN; ++b) {
    const int64_t j = j0 + wn0 + b * MF::BLK + jl;
    if (j >= g.N) continue;
    const int64_t cj = rmap(g.cn, j);
#pragma unroll
    for (int a = 0; a < FM; ++a) {
#pragma unroll
      for (int rr = 0; rr < MF::NACC; ++rr) {
        const int64_t i = i0 + wm0 + a * MF::BLK + MF::orow(lane, rr);
        if (i >= g.M) continue;
        double* p = C + rmap(g.cm, i) + cj;
        const double v = al * double(acc[a][b][rr]);
        *p = (g.beta == 0.0) ? v : v + g.beta * (*p);
      }
    }
  }
}

template <typename T, typename MF, int NS, int WGM, int WGN, int BK, int BM, int BN>
__global__ __launch_bounds__(64 * WGM * WGN) void gemm_dma_kernel(GemmArgs g) {
  gemm_dma_tile<T, MF, NS, WGM, WGN, BK, BM, BN>(g, blockIdx.x);
}

// the direct-to-LDS tile takes K-contiguous, 16-byte aligned operands without batch or split-K
static bool dma_ok(const GemmArgs& a, bool vec) { return vec && !a.b_ncontig && a.batch == 1 && a.k_split == 0; }

// Grouped launch: group gi owns blocks [start[gi], start[gi+1]); starts are
// multiples of 8 so a group's blocks keep the XCD round-robin of a plain launch.
template <int BM, int BN>
__device__ __forceinline__ int64_t group_of(const GemmGroup& gg, int64_t* local) {
  int gi = 0;
  while (gi + 1 < gg.ng && int64_t(blockIdx.x) >= gg.start[gi + 1]) ++gi;
  const GemmArgs& g = gg.g[gi];
  const int64_t l = int64_t(blockIdx.x) - gg.start[gi];
  const int64_t ntiles = ((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN);
  *local = l;
  return l < ntiles ? gi : -1;
}

template <typename T, typename MF, int BM, int BN, int WGM, int WGN, int KM, bool VEC>
__global__ __launch_bounds__(64 * WGM * WGN) void gemm_db_grouped_kernel(GemmGroup gg) {
  int64_t local = 0;
  const int64_t gi = group_of<BM, BN>(gg, &local);
  if (gi < 0) return;  // padding block of a group
  gemm_db_tile<T, MF, BM, BN, WGM, WGN, KM, VEC>(gg.g[gi], local);
}

template <typename T, typename MF, int NS, int WGM, int WGN, int BK, int BM, int BN>
__global__ __launch_bounds__(64 * WGM * WGN) void gemm_dma_grouped_kernel(GemmGroup gg) {
  int64_t local = 0;
  const int64_t gi = group_of<BM, BN>(gg, &local);
  if (gi < 0) return;
  gemm_dma_tile<T, MF, NS, WGM, WGN, BK, BM, BN>(gg.g[gi], local);
}

template <typename T, int BM, int BN, bool VEC>
__global__ __launch_bounds__(256) void gemm_grouped_kernel(GemmGroup gg) {
  int64_t local = 0;
  const int64_t gi = group_of<BM, BN>(gg, &local);
  if (gi < 0) return;
  gemm_tile<T, BM, BN, VEC, false>(gg.g[gi], local);
}

template <typename T, int BM, int BN, int WGM, int WGN, int KM = 1, typename MF = Mfma<T>>
static void launch_db(const GemmArgs& a, bool vec, hipStream_t s) {
  const int64_t tiles = ((a.M + BM - 1) / BM) * ((a.N + BN - 1) / BN);
  GFCC_CHECK(tiles < (int64_t(1) << 31) && a.batch < 65536, GFCC_E_ARG, "GEMM grid too large");
  GFCC_CHECK(!a.b_ncontig, GFCC_E_ARG, "double-buffered tiles need a K-contiguous B");
  dim3 grid(unsigned(tiles), 1, unsigned(a.batch));
  if (vec)
    hipLaunchKernelGGL((gemm_db_kernel<T, MF, BM, BN, WGM, WGN, KM, true>), grid, dim3(64 * WGM * WGN), 0, s, a);
  else
    hipLaunchKernelGGL((gemm_db_kernel<T, MF, BM, BN, WGM, WGN, KM, false>), grid, dim3(64 * WGM * WGN), 0, s, a);
  GFCC_HIP(hipGetLastError());
}

// 16-bit types take the 32x32x16 blocks, FP64 the 16x16x4 ones; BK in elements
template <typename T, int NS, int WGM, int WGN, int BK = 32, int BM = 256, int BN = 256>
static void launch_dma(const GemmArgs& a, hipStream_t s) {
  using MF = std::conditional_t<sizeof(T) == 2, typename Wide<T>::type, Mfma<T>>;
  const int64_t tiles = ((a.M + BM - 1) / BM) * ((a.N + BN - 1) / BN);
  GFCC_CHECK(tiles < (int64_t(1) << 31), GFCC_E_ARG, "GEMM grid too large");
  hipLaunchKernelGGL((gemm_dma_kernel<T, MF, NS, WGM, WGN, BK, BM, BN>), dim3(unsigned(tiles)), dim3(64 * WGM * WGN),
                     0, s, a);
  GFCC_HIP(hipGetLastError());
}
template <typename T, int NS, int WGM, int WGN, int BK = 32, int BM = 256, int BN = 256>
static void launch_dma_grouped(const GemmGroup& gg, hipStream_t s) {
  using MF = std::conditional_t<sizeof(T) == 2, typename Wide<T>::type, Mfma<T>>;
  hipLaunchKernelGGL((gemm_dma_grouped_kernel<T, MF, NS, WGM, WGN, BK, BM, BN>), dim3(unsigned(gg.start[gg.ng])),
                     dim3(64 * WGM * WGN), 0, s, gg);
  GFCC_HIP(hipGetLastError());
}

template <typename T, int BM, int BN>
static void launch(const GemmArgs& a, bool vec, hipStream_t s) {
  const int64_t tiles = ((a.M + BM - 1) / BM) * ((a.N + BN - 1) / BN);
  GFCC_CHECK(tiles < (int64_t(1) << 31) && a.batch < 65536, GFCC_E_ARG, "GEMM grid too large");
  dim3 grid(unsigned(tiles), 1, unsigned(a.batch));
  if (a.b_ncontig) {
    if (vec)
      hipLaunchKernelGGL((gemm_kernel<T, BM, BN, true, true>), grid, dim3(256), 0, s, a);
    else
      hipLaunchKernelGGL((gemm_kernel<T, BM, BN, false, true>), grid, dim3(256), 0, s, a);
  } else {
    if (vec)
      hipLaunchKernelGGL((gemm_kernel<T, BM, BN, true, false>), grid, dim3(256), 0, s, a);
    else
      hipLaunchKernelGGL((gemm_kernel<T, BM, BN, false, false>), grid, dim3(256), 0, s, a);
  }
  GFCC_HIP(hipGetLastError());
}

template <typename T>
static void dispatch(const GemmArgs& a, int cfg, bool vec, hipStream_t s) {
  switch (cfg) {
    case TILE_128x128: launch<T, 128, 128>(a, vec, s); break;
    case TILE_64x64: launch<T, 64, 64>(a, vec, s); break;
    case TILE_128x64: launch<T, 128, 64>(a, vec, s); break;
    case TILE_64x128: launch<T, 64, 128>(a, vec, s); break;
    case TILE_DB_128x128: launch_db<T, 128, 128, 2, 2>(a, vec, s); break;
    case TILE_DB_256x128: launch_db<T, 256, 128, 4, 2>(a, vec, s); break;
    case TILE_DB_128x256: launch_db<T, 128, 256, 2, 4>(a, vec, s); break;
    case TILE_DB_256x256: launch_db<T, 256, 256, 4, 2>(a, vec, s); break;
    // 32x32 MFMA blocks (BF16 and FP16; other types run the 16x16 kernel of the same tile)
    case TILE_DB32_256x256:
      if constexpr (Wide<T>::on) launch_db<T, 256, 256, 4, 2, 1, typename Wide<T>::type>(a, vec, s);
      else launch_db<T, 256, 256, 4, 2>(a, vec, s);
      break;
    case TILE_DB32_256x128:
      if constexpr (Wide<T>::on) launch_db<T, 256, 128, 4, 2, 1, typename Wide<T>::type>(a, vec, s);
      else launch_db<T, 256, 128, 4, 2>(a, vec, s);
      break;
    case TILE_DB32_128x128:
      if constexpr (Wide<T>::on) launch_db<T, 128, 128, 2, 2, 1, typename Wide<T>::type>(a, vec, s);
      else launch_db<T, 128, 128, 2, 2>(a, vec, s);
      break;
    // 16 waves of 64x64 (BF16, FP16): four waves per SIMD hide the global-load latency of the next K stage
    case TILE_DB32_256x256_W16:
      if constexpr (Wide<T>::on) launch_db<T, 256, 256, 4, 4, 1, typename Wide<T>::type>(a, vec, s);
      else launch_db<T, 256, 256, 4, 2>(a, vec, s);
      break;
    case TILE_DB_256x256_W16:
      if constexpr (Wide<T>::on) launch_db<T, 256, 256, 4, 4>(a, vec, s);
      else launch_db<T, 256, 256, 4, 2>(a, vec, s);
      break;
    case TILE_DMA3_256x256:
    case TILE_DMA4_256x256:
    case TILE_DMA3_256x256_W8:
    case TILE_DMA3_256x256_W8T:
    case TILE_DMA2K64_256x256:
      if constexpr (Wide<T>::on) {
        if (!dma_ok(a, vec)) launch_db<T, 256, 256, 4, 4, 1, typename Wide<T>::type>(a, vec, s);
        else if (cfg == TILE_DMA3_256x256) launch_dma<T, 3, 4, 4>(a, s);
        else if (cfg == TILE_DMA4_256x256) launch_dma<T, 4, 4, 4>(a, s);
        else if (cfg == TILE_DMA3_256x256_W8) launch_dma<T, 3, 2, 4>(a, s);
        else if (cfg == TILE_DMA3_256x256_W8T) launch_dma<T, 3, 4, 2>(a, s);
        else launch_dma<T, 2, 4, 4, 64>(a, s);
      } else {
        launch_db<T, 256, 256, 4, 2>(a, vec, s);
      }
      break;
    case TILE_DMA3_256x128:
    case TILE_DMA2_256x128:
      if constexpr (std::is_same_v<T, double>) {
        if (!dma_ok(a, vec)) launch_db<T, 256, 128, 4, 2>(a, vec, s);
        else if (cfg == TILE_DMA3_256x128) launch_dma<T, 3, 4, 2, 16, 256, 128>(a, s);
        else launch_dma<T, 2, 4, 2, 16, 256, 128>(a, s);
      } else if constexpr (std::is_same_v<T, float>) {
        if (!dma_ok(a, vec)) launch_db<T, 256, 128, 4, 2>(a, vec, s);
        else if (cfg == TILE_DMA3_256x128) launch_dma<T, 3, 4, 2, 32, 256, 128>(a, s);
        else launch_dma<T, 2, 4, 2, 32, 256, 128>(a, s);
      } else {
        launch_db<T, 256, 128, 4, 2>(a, vec, s);
      }
      break;
    case TILE_DMA2_128x256:
      if constexpr (std::is_same_v<T, double>) {
        if (!dma_ok(a, vec)) launch_db<T, 128, 256, 2, 4>(a, vec, s);
        else launch_dma<T, 2, 2, 4, 16, 128, 256>(a, s);
      } else {
        launch_db<T, 128, 256, 2, 4>(a, vec, s);
      }
      break;
    default: throw Error{GFCC_E_ARG, "bad tile config"};
  }
}

template <typename T, int BM, int BN, int WGM, int WGN, int KM = 1, typename MF = Mfma<T>>
static void launch_db_grouped(const GemmGroup& gg, bool vec, hipStream_t s) {
  dim3 grid(unsigned(gg.start[gg.ng]), 1, 1);
  if (vec)
    hipLaunchKernelGGL((gemm_db_grouped_kernel<T, MF, BM, BN, WGM, WGN, KM, true>), grid, dim3(64 * WGM * WGN), 0, s,
                       gg);
  else
    hipLaunchKernelGGL((gemm_db_grouped_kernel<T, MF, BM, BN, WGM, WGN, KM, false>), grid, dim3(64 * WGM * WGN), 0,
                       s, gg);
  GFCC_HIP(hipGetLastError());
}

template <typename T, int BM, int BN>
static void launch_grouped(const GemmGroup& gg, bool vec, hipStream_t s) {
  dim3 grid(unsigned(gg.start[gg.ng]), 1, 1);
  if (vec)
    hipLaunchKernelGGL((gemm_grouped_kernel<T, BM, BN, true>), grid, dim3(256), 0, s, gg);
  else
    hipLaunchKernelGGL((gemm_grouped_kernel<T, BM, BN, false>), grid, dim3(256), 0, s, gg);
  GFCC_HIP(hipGetLastError());
}

// tile sizes of a configuration
static void tile_dims(int cfg, int* bm, int* bn) {
  switch (cfg) {
    case TILE_128x128: case TILE_DB_128x128: case TILE_DB32_128x128: *bm = 128; *bn = 128; return;
    case TILE_64x64: *bm = 64; *bn = 64; return;
    case TILE_128x64: *bm = 128; *bn = 64; return;
    case TILE_64x128: *bm = 64; *bn = 128; return;
    case TILE_DB_256x128: case TILE_DB32_256x128: case TILE_DMA3_256x128: case TILE_DMA2_256x128:
      *bm = 256; *bn = 128; return;
    case TILE_DB_128x256: case TILE_DMA2_128x256: *bm = 128; *bn = 256; return;
    case TILE_DB_256x256: case TILE_DB32_256x256: case TILE_DB32_256x256_W16: case TILE_DB_256x256_W16:
    case TILE_DMA3_256x256: case TILE_DMA4_256x256: case TILE_DMA3_256x256_W8: case TILE_DMA3_256x256_W8T:
    case TILE_DMA2K64_256x256:
      *bm = 256; *bn = 256; return;
    default: throw Error{GFCC_E_ARG, "bad tile config"};
  }
}

template <typename T>
static void dispatch_grouped(const GemmGroup& gg, int cfg, bool vec, hipStream_t s) {
  switch (cfg) {
    case TILE_128x128: launch_grouped<T, 128, 128>(gg, vec, s); break;
    case TILE_64x64: launch_grouped<T, 64, 64>(gg, vec, s); break;
    case TILE_128x64: launch_grouped<T, 128, 64>(gg, vec, s); break;
    case TILE_64x128: launch_grouped<T, 64, 128>(gg, vec, s); break;
    case TILE_DB_128x128: launch_db_grouped<T, 128, 128, 2, 2>(gg, vec, s); break;
    case TILE_DB_256x128: launch_db_grouped<T, 256, 128, 4, 2>(gg, vec, s); break;
    case TILE_DB_128x256: launch_db_grouped<T, 128, 256, 2, 4>(gg, vec, s); break;
    case TILE_DB_256x256: launch_db_grouped<T, 256, 256, 4, 2>(gg, vec, s); break;
    case TILE_DB32_256x256:
      if constexpr (Wide<T>::on) launch_db_grouped<T, 256, 256, 4, 2, 1, typename Wide<T>::type>(gg, vec, s);
      else launch_db_grouped<T, 256, 256, 4, 2>(gg, vec, s);
      break;
    case TILE_DB32_256x128:
      if constexpr (Wide<T>::on) launch_db_grouped<T, 256, 128, 4, 2, 1, typename Wide<T>::type>(gg, vec, s);
      else launch_db_grouped<T, 256, 128, 4, 2>(gg, vec, s);
      break;
    case TILE_DB32_128x128:
      if constexpr (Wide<T>::on) launch_db_grouped<T, 128, 128, 2, 2, 1, typename Wide<T>::type>(gg, vec, s);
      else launch_db_grouped<T, 128, 128, 2, 2>(gg, vec, s);
      break;
    case TILE_DB32_256x256_W16:
      if constexpr (Wide<T>::on) launch_db_grouped<T, 256, 256, 4, 4, 1, typename Wide<T>::type>(gg, vec, s);
      else launch_db_grouped<T, 256, 256, 4, 2>(gg, vec, s);
      break;
    case TILE_DB_256x256_W16:
      if constexpr (Wide<T>::on) launch_db_grouped<T, 256, 256, 4, 4>(gg, vec, s);
      else launch_db_grouped<T, 256, 256, 4, 2>(gg, vec, s);
      break;
    case TILE_DMA3_256x256:
    case TILE_DMA4_256x256:
    case TILE_DMA3_256x256_W8:
    case TILE_DMA3_256x256_W8T:
    case TILE_DMA2K64_256x256:
      if constexpr (Wide<T>::on) {
        if (!vec) launch_db_grouped<T, 256, 256, 4, 4, 1, typename Wide<T>::type>(gg, vec, s);
        else if (cfg == TILE_DMA3_256x256) launch_dma_grouped<T, 3, 4, 4>(gg, s);
        else if (cfg == TILE_DMA4_256x256) launch_dma_grouped<T, 4, 4, 4>(gg, s);
        else if (cfg == TILE_DMA3_256x256_W8) launch_dma_grouped<T, 3, 2, 4>(gg, s);
        else if (cfg == TILE_DMA3_256x256_W8T) launch_dma_grouped<T, 3, 4, 2>(gg, s);
        else launch_dma_grouped<T, 2, 4, 4, 64>(gg, s);
      } else {
        launch_db_grouped<T, 256, 256, 4, 2>(gg, vec, s);
      }
      break;
    case TILE_DMA3_256x128:
    case TILE_DMA2_256x128:
      if constexpr (std::is_same_v<T, double>) {
        if (!vec) launch_db_grouped<T, 256, 128, 4, 2>(gg, vec, s);
        else if (cfg == TILE_DMA3_256x128) launch_dma_grouped<T, 3, 4, 2, 16, 256, 128>(gg, s);
        else launch_dma_grouped<T, 2, 4, 2, 16, 256, 128>(gg, s);
      } else if constexpr (std::is_same_v<T, float>) {
        if (!vec) launch_db_grouped<T, 256, 128, 4, 2>(gg, vec, s);
        else if (cfg == TILE_DMA3_256x128) launch_dma_grouped<T, 3, 4, 2, 32, 256, 128>(gg, s);
        else launch_dma_grouped<T, 2, 4, 2, 32, 256, 128>(gg, s);
      } else {
        launch_db_grouped<T, 256, 128, 4, 2>(gg, vec, s);
      }
      break;
    case TILE_DMA2_128x256:
      if constexpr (std::is_same_v<T, double>) {
        if (!vec) launch_db_grouped<T, 128, 256, 2, 4>(gg, vec, s);
        else launch_dma_grouped<T, 2, 2, 4, 16, 128, 256>(gg, s);
      } else {
        launch_db_grouped<T, 128, 256, 2, 4>(gg, vec, s);
      }
      break;
    default: throw Error{GFCC_E_ARG, "bad tile config"};
  }
}

static bool aligned_map(const RowMap& m, int64_t epc) {
  return (m.hi % epc) == 0 && (m.lo % epc) == 0;
}

// C(i,j) = alpha * sum_z part[z][i][j] + beta * C(i,j)
__global__ void splitk_reduce_kernel(const double* __restrict__ part, int slices, int64_t M, int64_t N, double* C,
                                     RowMap cm, RowMap cn, double alpha, double beta, const double* alpha_dev) {
  const int64_t MN = M * N;
  if (alpha_dev) alpha *= *alpha_dev;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < MN; t += int64_t(gridDim.x) * blockDim.x) {
    double acc = 0.0;
    for (int z = 0; z < slices; ++z) acc += part[z * MN + t];
    const int64_t i = t / N, j = t % N;
    double* p = C + rmap(cm, i) + rmap(cn, j);
    const double v = alpha * acc;
    *p = (beta == 0.0) ? v : v + beta * (*p);
  }
}

int splitk_slices(int64_t M, int64_t N, int64_t K) {
  const int cfg = gemm_default_cfg(M, N, K);
  const int64_t bm = (cfg == TILE_128x128 || cfg == TILE_128x64) ? 128 : 64;
  const int64_t bn = (cfg == TILE_128x128 || cfg == TILE_64x128) ? 128 : 64;
  const int64_t tiles = ((M + bm - 1) / bm) * ((N + bn - 1) / bn);
  if (tiles >= 256 || K < 2048) return 1;
  int64_t sl = std::min<int64_t>((512 + tiles - 1) / tiles, K / 1024);
  return int(std::max<int64_t>(1, std::min<int64_t>(sl, 256)));
}

void gemm_splitk(Prec p, const GemmArgs& a, int slices, double* part, hipStream_t s) {
  if (a.M <= 0 || a.N <= 0) return;
  GemmArgs g = a;
  const int64_t epc = (p == Prec::F64) ? 2 : (p == Prec::F32 ? 4 : 8);
  g.k_split = round_up((a.K + slices - 1) / slices, 8 * epc);
  const int nsl = int((a.K + g.k_split - 1) / g.k_split);
  g.batch = nsl;
  g.C = part;
  g.cm = lin(a.N);
  g.cn = lin(1);
  g.cz = lin(a.M * a.N);
  g.alpha = 1.0;
  g.beta = 0.0;
  g.alpha_dev = nullptr;
  gemm(p, g, gemm_default_cfg(a.M, a.N, a.K), s);
  const int64_t MN = a.M * a.N;
  const unsigned nb = unsigned(std::min<int64_t>((MN + 255) / 256, 4096));
  hipLaunchKernelGGL(splitk_reduce_kernel, dim3(nb), dim3(256), 0, s, part, nsl, a.M, a.N, a.C, a.cm, a.cn,
                     a.alpha, a.beta, a.alpha_dev);
  GFCC_HIP(hipGetLastError());
}

void gemm_auto(Prec p, const GemmArgs& a, Scratch& scr, int scr_slot, hipStream_t s) {
  const int sl = (a.batch == 1) ? splitk_slices(a.M, a.N, a.K) : 1;
  if (sl <= 1) {
    gemm(p, a, gemm_default_cfg(a.M, a.N, a.K), s);
    return;
  }
  double* part = scr.get(scr_slot, int64_t(sl) * a.M * a.N, s);
  gemm_splitk(p, a, sl, part, s);
}

const char* tile_name(int cfg) {
  static const char* n[] = {"128x128", "64x64", "128x64", "64x128", "db128x128", "db256x128", "db128x256",
                            "db256x256", "db32_256x256", "db32_256x128", "db32_128x128", "db32_256x256w16", "db256x256w16",
                            "dma3_256x256", "dma4_256x256", "dma3_256x256w8", "dma3_256x256w8t", "dma2k64_256x256", "dma3_256x128", "dma2_256x128", "dma2_128x256"};
  return (cfg >= 0 && cfg < N_TILE_CFG) ? n[cfg] : "?";
}

// Tiles for large K-contiguous products when no tuned entry exists (the fastest on the ring
// shapes): the 256x128 tile that loads straight into two (FP64) or three (FP32) LDS stages, and
// in BF16 and FP16 the 16-wave 256x256 tile with two LDS stages of K = 64 filled the same way.
int gemm_big_cfg(Prec p, int64_t M, int64_t N, int64_t K) {
  if (M >= 2048 && N >= 2048 && K >= 256) {
    if (p == Prec::BF16 || p == Prec::F16) return TILE_DMA2K64_256x256;
    return p == Prec::F64 ? TILE_DMA2_256x128 : TILE_DMA3_256x128;
  }
  return gemm_default_cfg(M, N, K);
}

int gemm_default_cfg(int64_t M, int64_t N, int64_t K) {
  (void)K;
  const int64_t big = (M >= 512 && N >= 512) ? 1 : 0;
  if (big) return TILE_128x128;
  if (M >= 128 && N < 128) return TILE_128x64;
  if (N >= 128 && M < 128) return TILE_64x128;
  return TILE_64x64;
}

void gemm(Prec p, const GemmArgs& a, int cfg, hipStream_t s) {
  if (a.M <= 0 || a.N <= 0 || a.batch <= 0) return;
  GFCC_CHECK(a.K >= 0, GFCC_E_ARG, "negative K");
  GFCC_CHECK(a.am.div > 0 && a.bm.div > 0 && a.cm.div > 0 && a.cn.div > 0, GFCC_E_ARG, "bad row map");
  const int64_t esz = (p == Prec::F64) ? 8 : (p == Prec::F32 ? 4 : 2);
  const int64_t epc = 16 / esz;
  const bool vec = aligned_map(a.am, epc) && aligned_map(a.bm, epc) && aligned_map(a.az, epc) &&
                   aligned_map(a.bz, epc) && (reinterpret_cast<uintptr_t>(a.A) % 16 == 0) &&
                   (reinterpret_cast<uintptr_t>(a.B) % 16 == 0) && (a.k_split % epc == 0);
  switch (p) {
    case Prec::F64: dispatch<double>(a, cfg, vec, s); break;
    case Prec::F32: dispatch<float>(a, cfg, vec, s); break;
    case Prec::BF16: dispatch<__bf16>(a, cfg, vec, s); break;
    case Prec::F16: dispatch<_Float16>(a, cfg, vec, s); break;
  }
}

void gemm_grouped(Prec p, const GemmArgs* a, int ng, int cfg, hipStream_t s) {
  GFCC_CHECK(ng >= 0 && ng <= MAX_GEMM_GROUPS, GFCC_E_ARG, "too many GEMM groups");
  const int64_t esz = (p == Prec::F64) ? 8 : (p == Prec::F32 ? 4 : 2);
  const int64_t epc = 16 / esz;
  int bm = 0, bn = 0;
  tile_dims(cfg, &bm, &bn);
  GemmGroup gg;
  gg.ng = 0;
  gg.start[0] = 0;
  bool vec = true;
  for (int i = 0; i < ng; ++i) {
    const GemmArgs& x = a[i];
    if (x.M <= 0 || x.N <= 0) continue;
    GFCC_CHECK(x.K >= 0 && x.batch == 1 && x.k_split == 0 && !x.b_ncontig, GFCC_E_ARG,
               "grouped GEMM: batch 1, no split-K, K-contiguous B");
    GFCC_CHECK(x.am.div > 0 && x.bm.div > 0 && x.cm.div > 0 && x.cn.div > 0, GFCC_E_ARG, "bad row map");
    vec = vec && aligned_map(x.am, epc) && aligned_map(x.bm, epc) && (reinterpret_cast<uintptr_t>(x.A) % 16 == 0) &&
          (reinterpret_cast<uintptr_t>(x.B) % 16 == 0);
    const int64_t tiles = ((x.M + bm - 1) / bm) * ((x.N + bn - 1) / bn);
    gg.g[gg.ng] = x;
    gg.start[gg.ng + 1] = gg.start[gg.ng] + (tiles + 7) / 8 * 8;
    gg.ng += 1;
  }
  if (gg.ng == 0) return;
  GFCC_CHECK(gg.start[gg.ng] < (int64_t(1) << 31), GFCC_E_ARG, "GEMM grid too large");
  switch (p) {
    case Prec::F64: dispatch_grouped<double>(gg, cfg, vec, s); break;
    case Prec::F32: dispatch_grouped<float>(gg, cfg, vec, s); break;
    case Prec::BF16: dispatch_grouped<__bf16>(gg, cfg, vec, s); break;
    case Prec::F16: dispatch_grouped<_Float16>(gg, cfg, vec, s); break;
  }
}

}  // namespace gfcc

// Tile autotuner for the sigma GEMMs.  The paper's tensor layer relies on a
// few tens of kernels tuned by vendor libraries, code generation plus
// autotuning, or hand tuning (Tensor Algebra for Many-body Methods); here every
// tile configuration of the MFMA GEMM is timed with HIP events on the sigma's
// GEMM shapes (ring: M = vector rows, N = K = o*v; hole-hole ladder; three-body
// + 2h1p<-1h) and the fastest is kept per (precision, M, N, K).  Results
// persist in a small JSON file.
#include <cstdlib>
#include <cmath>
#include <cstdio>
#include <fstream>
#include <sstream>
#include <string>

#include "ctx.h"

namespace gfcc {

static std::string tune_key(Prec p, int64_t M, int64_t N, int64_t K) {
  char key[96];
  snprintf(key, sizeof key, "%d:%lld:%lld:%lld", int(p), (long long)M, (long long)N, (long long)K);
  return key;
}

void tune_load(gfcc_ctx* c, const char* path) {
  if (!path) return;
  std::ifstream f(path);
  if (!f) return;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string t = ss.str();
  // entries look like {"key": "2:10240:8000:8000", "cfg": 5, ...}
  size_t pos = 0;
  while ((pos = t.find("\"key\": \"", pos)) != std::string::npos) {
    pos += 8;
    const size_t e = t.find('"', pos);
    if (e == std::string::npos) break;
    const std::string key = t.substr(pos, e - pos);
    const size_t cp = t.find("\"cfg\": ", e);
    if (cp == std::string::npos) break;
    const int cfg = std::atoi(t.c_str() + cp + 7);
    // an entry written by a build with another tile table names a different tile: skip it
    const size_t np = t.find("\"name\": \"", cp);
    const size_t nxt = t.find("\"key\": \"", cp);
    bool same_tile = false;
    if (cfg >= 0 && cfg < N_TILE_CFG && np != std::string::npos && (nxt == std::string::npos || np < nxt)) {
      const size_t ne = t.find('"', np + 9);
      same_tile = ne != std::string::npos && t.compare(np + 9, ne - (np + 9), tile_name(cfg)) == 0;
    }
    if (same_tile) {
      c->tuned[key] = cfg;
      const size_t mp = t.find("\"ms\": ", cp);
      const size_t next = t.find("\"key\": \"", cp);
      if (mp != std::string::npos && (next == std::string::npos || mp < next))
        c->tuned_ms[key] = float(std::atof(t.c_str() + mp + 6));
    }
    pos = cp;
  }
}

void tune_save(gfcc_ctx* c, const char* path) {
  if (!path) return;
  std::ofstream f(path);
  if (!f) return;
  f << "{\"entries\": [\n";
  size_t k = 0;
  for (const auto& kv : c->tuned) {
    f << "  {\"key\": \"" << kv.first << "\", \"cfg\": " << kv.second << ", \"name\": \"" << tile_name(kv.second)
      << "\", \"ms\": " << c->tuned_ms[kv.first] << "}" << (++k < c->tuned.size() ? "," : "") << "\n";
  }
  f << "]}\n";
}

template <typename T>
__global__ void fill_kernel(T* p, int64_t n, double val) {
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n; t += int64_t(gridDim.x) * blockDim.x)
    p[t] = T(float(val));
}

static void fill(Prec p, void* dst, int64_t n, double val, hipStream_t s) {
  const dim3 g(unsigned(std::min<int64_t>((n + 255) / 256, 4096)));
  switch (p) {
    case Prec::F64: hipLaunchKernelGGL(fill_kernel<double>, g, dim3(256), 0, s, static_cast<double*>(dst), n, val); break;
    case Prec::F32: hipLaunchKernelGGL(fill_kernel<float>, g, dim3(256), 0, s, static_cast<float*>(dst), n, val); break;
    case Prec::BF16: hipLaunchKernelGGL(fill_kernel<__bf16>, g, dim3(256), 0, s, static_cast<__bf16*>(dst), n, val); break;
    case Prec::F16: hipLaunchKernelGGL(fill_kernel<_Float16>, g, dim3(256), 0, s, static_cast<_Float16*>(dst), n, val); break;
  }
  GFCC_HIP(hipGetLastError());
}

// Time every tile configuration on C[M][N] = A[M][K] B[N][K]^T (both operands
// K-contiguous, filled with a constant) and keep the fastest.
static void tune_shape(gfcc_ctx* c, Prec p, int64_t M, int64_t N, int64_t K, hipStream_t s) {
  const std::string key = tune_key(p, M, N, K);
  if (c->tuned.count(key) || M <= 0 || N <= 0 || K <= 0) return;
  const int64_t esz = (p == Prec::F64) ? 8 : (p == Prec::F32 ? 4 : 2);
  const int64_t ldk = round_up(K, 8);
  DBuf a, b, cbuf;
  a.ensure(size_t(M * ldk * esz), s);
  b.ensure(size_t(N * ldk * esz), s);
  cbuf.ensure(size_t(M * N) * 8, s);
  fill(p, a.p, M * ldk, 0.5, s);
  fill(p, b.p, N * ldk, 0.25, s);
  GemmArgs g;
  g.A = a.p;
  g.am = lin(ldk);
  g.B = b.p;
  g.bm = lin(ldk);
  g.C = cbuf.as<double>();
  g.cm = lin(N);
  g.cn = lin(1);
  g.M = M;
  g.N = N;
  g.K = K;
  hipEvent_t e0, e1;
  GFCC_HIP(hipEventCreate(&e0));
  GFCC_HIP(hipEventCreate(&e1));
  int best = gemm_default_cfg(M, N, K);
  float best_ms = 1e30f;
  for (int cfg = 0; cfg < N_TILE_CFG; ++cfg) {
    gemm(p, g, cfg, s);  // warm-up
    GFCC_HIP(hipEventRecord(e0, s));
    const int reps = 3;
    for (int r = 0; r < reps; ++r) gemm(p, g, cfg, s);
    GFCC_HIP(hipEventRecord(e1, s));
    GFCC_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    GFCC_HIP(hipEventElapsedTime(&ms, e0, e1));
    ms /= float(reps);
    if (std::getenv("GFCC_VERBOSE"))
      std::fprintf(stderr, "[gfcc] tune prec %d M %lld N %lld K %lld %-18s %9.3f ms %8.1f TFLOP/s\n", int(p),
                   (long long)M, (long long)N, (long long)K, tile_name(cfg), double(ms),
                   2.0 * double(M) * double(N) * double(K) / (double(ms) * 1e9));
    if (ms < 0.99f * best_ms) {  // a later configuration must win by more than 1% (stable choice)
      best_ms = ms;
      best = cfg;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->tuned[key] = best;
  c->tuned_ms[key] = best_ms;
}

void tune_ring(gfcc_ctx* c, Prec p, int64_t P, hipStream_t s) {
  if (p != Prec::F64) build_lowprec(c, p == Prec::BF16 ? 1 : (p == Prec::F16 ? 2 : 0), s);
  tune_shape(c, p, P * c->o, c->ov, c->k2, s);  // ring, first product (K = [Wovvo | Wovov])
  tune_shape(c, p, P * c->o, c->ov, c->ov, s);  // ring, second product
  tune_shape(c, p, c->oo, P * c->v, c->oo, s);  // hole-hole ladder
  tune_shape(c, p, P * c->o, c->Q, c->kp, s);   // three-body U
  tune_shape(c, p, P, c->oov, c->o, s);         // 2h1p <- 1h
}

// GFCC_TILE_<PREC> (FP64, FP32, BF16, FP16) = a tile name forces that tile for every product that
// would otherwise take a tuned or default large tile of that precision (tests and tuning studies)
static int forced_cfg(Prec p) {
  static const char* var[4] = {"GFCC_TILE_FP64", "GFCC_TILE_FP32", "GFCC_TILE_BF16", "GFCC_TILE_FP16"};
  const char* v = std::getenv(var[int(p)]);
  if (!v || !*v) return -1;
  for (int cfg = 0; cfg < N_TILE_CFG; ++cfg)
    if (std::string(v) == tile_name(cfg)) return cfg;
  return -1;
}

int tuned_cfg(gfcc_ctx* c, Prec p, int64_t M, int64_t N, int64_t K) {
  if (forced_cfg(p) >= 0) return forced_cfg(p);
  const std::string key = tune_key(p, M, N, K);
  auto it = c->tuned.find(key);
  if (it != c->tuned.end()) return it->second;
  // closest tuned shape with the same precision and K (within a factor 4 overall)
  double best = std::log(4.0);
  int cfg = gemm_big_cfg(p, M, N, K);
  for (const auto& kv : c->tuned) {
    int pp = 0;
    long long m2 = 0, n2 = 0, k2 = 0;
    if (std::sscanf(kv.first.c_str(), "%d:%lld:%lld:%lld", &pp, &m2, &n2, &k2) != 4) continue;
    if (pp != int(p) || k2 != K || m2 <= 0 || n2 <= 0) continue;
    const double d = std::fabs(std::log(double(M) / double(m2))) + std::fabs(std::log(double(N) / double(n2)));
    if (d <= best) {
      best = d;
      cfg = kv.second;
    }
  }
  return cfg;
}

}  // namespace gfcc

// Tile autotuner for the ring GEMMs.  The paper's tensor layer relies on a
// few tens of kernels tuned by vendor libraries, code generation plus
// autotuning, or hand tuning (Tensor Algebra for Many-body Methods); here every
// tile configuration of the MFMA GEMM is timed with HIP events on the actual
// ring-GEMM shape (M = vector rows, N = K = o*v) and the fastest is kept per
// (precision, M, N, K).  Results persist in a small JSON file.
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
    if (cfg >= 0 && cfg < N_TILE_CFG) {
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

// Time all tile configurations for the ring GEMM with P planes in precision p.
void tune_ring(gfcc_ctx* c, Prec p, int64_t P, hipStream_t s) {
  const int64_t M = P * c->o, N = c->ov, K = c->ov;
  const std::string key = tune_key(p, M, N, K);
  if (c->tuned.count(key)) return;
  const int64_t esz = (p == Prec::F64) ? 8 : (p == Prec::F32 ? 4 : 2);
  if (p != Prec::F64) build_lowprec(c, p == Prec::BF16 ? 1 : 0, s);
  DBuf a, cbuf;
  a.ensure(size_t(M) * K * esz, s);
  cbuf.ensure(size_t(M) * N * 8, s);
  const void* B = (p == Prec::F64) ? c->X1.p : (p == Prec::F32 ? c->lp[0].X1.p : c->lp[1].X1.p);
  GemmArgs g;
  g.A = a.p;
  g.am = lin(K);
  g.B = B;
  g.bm = lin(c->kp);
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
    if (ms < best_ms) {
      best_ms = ms;
      best = cfg;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->tuned[key] = best;
  c->tuned_ms[key] = best_ms;
}

}  // namespace gfcc

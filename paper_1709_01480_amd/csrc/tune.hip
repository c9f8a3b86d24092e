// Autotuner: picks the spreading tile edge and, when the caller leaves the
// Ewald split free, the cutoff cell count n_box (r_c = L / n_box) and the grid
// it implies, by timing the single-layer matvec of the caller's configuration
// on the current device.  Choices are cached in a JSON-lines file keyed by the
// device, the precision and the problem, so a later context of the same
// problem takes them without timing.
//
// Cache line format (one JSON object per line; the last line of a key wins):
//   {"key": "<key>", "n_box": 201, "grid_M": 2048, "tile": 32, "ms": 0.298}
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "ctx.h"

namespace fbim {
namespace {

std::mutex g_cache_mutex;

struct Choice {
  int n_box = 0, grid_M = 0, tile = 0;
  double ms = 0.0;
};

// the integer after "\"name\":" in line, or -1
long json_int(const char *line, const char *name) {
  char pat[64];
  std::snprintf(pat, sizeof pat, "\"%s\":", name);
  const char *p = std::strstr(line, pat);
  if (!p) return -1;
  p += std::strlen(pat);
  char *end = nullptr;
  const long v = std::strtol(p, &end, 10);
  return end == p ? -1 : v;
}

double json_double(const char *line, const char *name) {
  char pat[64];
  std::snprintf(pat, sizeof pat, "\"%s\":", name);
  const char *p = std::strstr(line, pat);
  if (!p) return -1.0;
  p += std::strlen(pat);
  char *end = nullptr;
  const double v = std::strtod(p, &end);
  return end == p ? -1.0 : v;
}

// last well-formed line whose key equals `key` exactly
bool cache_find(const char *path, const std::string &key, Choice &out) {
  FILE *f = std::fopen(path, "r");
  if (!f) return false;
  const std::string want = "{\"key\": \"" + key + "\",";
  bool found = false;
  std::vector<char> buf(1 << 16);
  while (std::fgets(buf.data(), (int)buf.size(), f)) {
    const char *line = buf.data();
    if (std::strncmp(line, want.c_str(), want.size()) != 0) continue;
    Choice c;
    c.n_box = (int)json_int(line, "n_box");
    c.grid_M = (int)json_int(line, "grid_M");
    c.tile = (int)json_int(line, "tile");
    c.ms = json_double(line, "ms");
    if (c.n_box < 3 || c.grid_M < 2 || c.tile < 1) continue;  // malformed: ignored
    out = c;
    found = true;
  }
  std::fclose(f);
  return found;
}

bool cache_append(const char *path, const std::string &key, const Choice &c) {
  FILE *f = std::fopen(path, "a");
  if (!f) return false;
  const int n = std::fprintf(f, "{\"key\": \"%s\", \"n_box\": %d, \"grid_M\": %d, \"tile\": %d, \"ms\": %.6g}\n",
                             key.c_str(), c.n_box, c.grid_M, c.tile, c.ms);
  return std::fclose(f) == 0 && n > 0;
}

std::string problem_key(const fbim_ctx *c, uint32_t what) {
  hipDeviceProp_t prop{};
  std::string arch = "unknown";
  int cus = 0;
  if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) {
    arch = prop.gcnArchName;
    arch = arch.substr(0, arch.find(':'));
    cus = prop.multiProcessorCount;
  }
  // nodes per body of every shape with its body count
  std::vector<int> count(c->shapes.size(), 0);
  for (int s : c->h_shape) ++count[s];
  std::string shapes;
  for (size_t s = 0; s < c->shapes.size(); ++s)
    if (count[s]) shapes += (shapes.empty() ? "" : "+") + std::to_string(c->shapes[s].h.n_p) + "x" +
                            std::to_string(count[s]);
  char buf[512];
  std::snprintf(buf, sizeof buf,
                "arch=%s:cu=%d|prec=%d|N=%d|bodies=%s|L=%.9g|eps=%.3g|order=%d|M=%d|nbox=%d|xi=%.9g|P=%d|what=%u",
                arch.c_str(), cus, c->p.precision, c->N, shapes.c_str(), c->p.L, c->p.tol_ewald, c->p.alpert_order,
                c->p.grid_M, c->p.n_box, c->p.xi, c->p.P, what);
  return buf;
}

// a context with the parameters p and the configuration (shapes, bodies) of c
fbim_status trial_ctx(const fbim_ctx *c, const fbim_params &p, fbim_ctx **out) {
  fbim_params q = p;
  fbim_status st = fbim_create(&q, out);
  if (st != FBIM_OK) return st;
  fbim_set_stream(*out, c->stream);
  for (auto &sh : c->shapes) {
    int32_t id = 0;
    st = fbim_add_shape(*out, sh.h.n_p, sh.h.ref_xy.data(), &id);
    if (st != FBIM_OK) break;  // including r_Alpert / r_c above 0.6: not a candidate
  }
  if (st == FBIM_OK) st = fbim_set_bodies(*out, c->n, c->h_shape.data(), c->h_q.data(), c->h_theta.data());
  if (st != FBIM_OK) {
    fbim_destroy(*out);
    *out = nullptr;
  }
  return st;
}

// median time of `reps` single-layer matvecs (after two untimed ones), HIP events
// on the trial context's stream
fbim_status time_matvec(fbim_ctx *t, const double *mu, double *out, int reps, double &ms) {
  for (int i = 0; i < 2; ++i) STCHK(fbim_apply_M(t, mu, out, FBIM_PART_ALL));
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return FBIM_EDEVICE;
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return FBIM_EDEVICE;
  }
  std::vector<float> ts;
  fbim_status st = FBIM_OK;
  for (int i = 0; i < reps && st == FBIM_OK; ++i) {
    hipEventRecord(e0, t->stream);
    st = fbim_apply_M(t, mu, out, FBIM_PART_ALL);
    hipEventRecord(e1, t->stream);
    if (hipEventSynchronize(e1) != hipSuccess) st = FBIM_EDEVICE;
    float v = 0.f;
    hipEventElapsedTime(&v, e0, e1);
    ts.push_back(v);
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (st != FBIM_OK) return st;
  std::sort(ts.begin(), ts.end());
  ms = ts[ts.size() / 2];
  return FBIM_OK;
}

// tiles the parameter rule accepts for grid M and support P (at most 32)
std::vector<int> tile_candidates(int M, int P) {
  std::vector<int> out;
  for (int t = 32; t >= std::max(4, (P - 1) / 2); --t)
    if (M % t == 0 && M / t >= 3) out.push_back(t);
  return out;
}

}  // namespace
}  // namespace fbim

using namespace fbim;

extern "C" {

int32_t fbim_autotune_lookup(const char *cache_path, const char *key, int32_t *n_box, int32_t *grid_M,
                             int32_t *tile) {
  if (!cache_path || !key) return 0;
  Choice c;
  std::lock_guard<std::mutex> lk(g_cache_mutex);
  if (!cache_find(cache_path, key, c)) return 0;
  if (n_box) *n_box = c.n_box;
  if (grid_M) *grid_M = c.grid_M;
  if (tile) *tile = c.tile;
  return 1;
}

fbim_status fbim_autotune_key(const fbim_ctx *c, uint32_t what, char *buf, int32_t len) {
  if (!c || !buf || len <= 0) return FBIM_EINVAL;
  const std::string k = problem_key(c, what);
  if ((int32_t)k.size() >= len) return FBIM_EINVAL;
  std::memcpy(buf, k.c_str(), k.size() + 1);
  return FBIM_OK;
}

fbim_status fbim_autotune(fbim_ctx *c, uint32_t what, const char *cache_path, fbim_params *out,
                          fbim_tune_report *rep) {
  if (!c || !out) return FBIM_EINVAL;
  if (!c->have_bodies) return fail(c, FBIM_EINVAL, "autotune needs a configuration (fbim_set_bodies)");
  if (what == 0 || (what & ~(uint32_t)(FBIM_TUNE_TILE | FBIM_TUNE_SPLIT)))
    return fail(c, FBIM_EINVAL, "invalid tuning set");
  const bool split = (what & FBIM_TUNE_SPLIT) != 0;
  if (split && (c->p.grid_M != 0 || c->p.xi != 0.0 || c->p.n_box == 0))
    return fail(c, FBIM_EINVAL, "FBIM_TUNE_SPLIT needs n_box given and grid_M, xi left to the parameter rule");
  fbim_tune_report r{};
  const std::string key = problem_key(c, what);
  fbim_params base = c->p;
  Choice best;
  {
    std::lock_guard<std::mutex> lk(g_cache_mutex);
    if (cache_path && cache_find(cache_path, key, best)) {
      *out = base;
      out->n_box = best.n_box;
      out->grid_M = best.grid_M;
      out->tile = best.tile;
      r.from_cache = 1;
      r.ms_best = best.ms;
      r.ms_default = -1.0;
      if (rep) *rep = r;
      return FBIM_OK;
    }
  }
  // probe vector: a fixed pattern, no randomness needed for timing
  const size_t n2 = 2 * (size_t)c->N;
  double *mu = nullptr, *o = nullptr;
  if (hipMalloc((void **)&mu, n2 * sizeof(double)) != hipSuccess) return fail(c, FBIM_EDEVICE, "hipMalloc failed");
  if (hipMalloc((void **)&o, n2 * sizeof(double)) != hipSuccess) {
    hipFree(mu);
    return fail(c, FBIM_EDEVICE, "hipMalloc failed");
  }
  fbim_status st = launch_fill(n2, 1.0, mu, c->stream) == hipSuccess ? FBIM_OK : FBIM_EDEVICE;
  // candidate splits: the caller's n_box scaled, each with the grid of the parameter
  // rule and the next power of two (the fused transform path)
  std::vector<std::pair<int, int>> splits;  // (n_box, grid_M)
  if (split) {
    const double f[] = {0.6, 0.75, 0.9, 1.0, 1.15, 1.3};
    for (double s : f) {
      const int nb = std::max(3, (int)std::lround(c->p.n_box * s));
      fbim_params q = base;
      q.n_box = nb;
      q.grid_M = 0;
      q.tile = 0;
      fbim_derived d{};
      if (fbim_derive_params(&q, &d) != FBIM_OK) continue;
      int p2 = 64;
      while (p2 < d.grid_M) p2 *= 2;
      for (int M : {d.grid_M, p2})
        if (std::find(splits.begin(), splits.end(), std::make_pair(nb, M)) == splits.end())
          splits.push_back({nb, M});
    }
  } else {
    splits.push_back({c->d.n_box, c->d.M});
  }
  double ms_default = -1.0;
  {
    double ms = 0.0;
    if (st == FBIM_OK && time_matvec(c, mu, o, 5, ms) == FBIM_OK) ms_default = ms;
  }
  best.ms = -1.0;
  for (auto &sp : splits) {
    if (st != FBIM_OK) break;
    std::vector<int> tiles;
    if (what & FBIM_TUNE_TILE) {
      fbim_params q = base;
      q.n_box = sp.first;
      q.grid_M = sp.second;
      q.xi = 0.0;
      q.tile = 0;
      fbim_derived d{};
      if (fbim_derive_params(&q, &d) != FBIM_OK) continue;
      tiles = tile_candidates(d.grid_M, d.P);
    } else {
      tiles.push_back(split ? 0 : c->d.tile);
    }
    for (int t : tiles) {
      fbim_params q = base;
      q.n_box = sp.first;
      q.grid_M = sp.second;
      q.xi = split ? 0.0 : base.xi;
      q.tile = t;
      fbim_ctx *tc = nullptr;
      if (trial_ctx(c, q, &tc) != FBIM_OK) continue;  // not admissible (accuracy rule, tile rule)
      double ms = 0.0;
      const fbim_status ts = time_matvec(tc, mu, o, 5, ms);
      fbim_derived d{};
      fbim_get_derived(tc, &d);
      fbim_destroy(tc);
      if (ts != FBIM_OK) continue;
      ++r.candidates;
      if (best.ms < 0 || ms < best.ms) {
        best.ms = ms;
        best.n_box = d.n_box;
        best.grid_M = d.grid_M;
        best.tile = d.tile;
      }
    }
  }
  hipFree(mu);
  hipFree(o);
  if (st != FBIM_OK) return fail(c, st, "autotune: device error");
  if (best.ms < 0) return fail(c, FBIM_EINVAL, "autotune: no admissible candidate");
  *out = base;
  out->n_box = best.n_box;
  out->grid_M = best.grid_M;
  out->tile = best.tile;
  if (split) out->xi = 0.0;
  r.ms_best = best.ms;
  r.ms_default = ms_default;
  if (cache_path) {
    std::lock_guard<std::mutex> lk(g_cache_mutex);
    if (!cache_append(cache_path, key, best)) r.cache_error = 1;
  }
  if (rep) *rep = r;
  return FBIM_OK;
}

}  // extern "C"

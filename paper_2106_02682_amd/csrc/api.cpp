// C ABI of libvemb (declared in include/vemb.h): problem lifetime, the
// iteration schedule of Algorithm 6 on one stream, diagnostics and state I/O.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <filesystem>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "alloc.h"
#include "polar.h"
#include "problem.h"
#include "sign_batched.h"
#include "tile_map.h"

namespace vemb {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

}  // namespace vemb

using namespace vemb;



namespace vemb {
namespace {
std::mutex g_alloc_mu;
Allocator g_alloc;
int g_live_objects = 0;
}  // namespace

Allocator current_allocator() {
  std::lock_guard<std::mutex> lock(g_alloc_mu);
  return g_alloc;
}
void object_created() {
  std::lock_guard<std::mutex> lock(g_alloc_mu);
  ++g_live_objects;
}
void object_destroyed() {
  std::lock_guard<std::mutex> lock(g_alloc_mu);
  --g_live_objects;
}

int fail(int code, const std::string& msg) {
  set_error(msg);
  return code;
}

int hip_rc(hipError_t e, const char* what) {
  if (e == hipSuccess) return VEMB_OK;
  return fail(VEMB_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}
}  // namespace vemb

namespace {

template <typename T>
int dalloc(vemb_problem* p, T** ptr, size_t count) {
  const size_t bytes = count == 0 ? 16 : count * sizeof(T);
  void* raw = p->mem.get(bytes);
  if (!raw) return fail(VEMB_E_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  *ptr = static_cast<T*>(raw);
  return VEMB_OK;
}


int upload_initial_state(vemb_problem* p) {
  const int m = p->g.m, n = p->g.n, M = p->g.M, P = p->P, k = p->n_op;
  std::vector<double> X((size_t)M * k * k, 0.0);
  for (int i = 0; i < k; ++i) X[(size_t)i * k + i] = 1.0;  // X_00 = I, X_0d = 0
  std::vector<double> rho0((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i) rho0[(size_t)i * m + i] = 1.0 / m;
  std::vector<double> rt((size_t)P * n * n, 0.0);
  for (int d = 0; d < P; ++d)
    for (int i = 0; i < n; ++i) rt[(size_t)d * n * n + (size_t)i * n + i] = 1.0 / n;
  hipStream_t s = p->stream;
  VEMB_TRY(hip_rc(hipMemcpyAsync(p->a.X, X.data(), X.size() * 8, hipMemcpyHostToDevice, s), "upload X"));
  VEMB_TRY(hip_rc(hipMemcpyAsync(p->a.rho0, rho0.data(), rho0.size() * 8, hipMemcpyHostToDevice, s), "upload rho0"));
  VEMB_TRY(hip_rc(hipMemcpyAsync(p->a.rho_t, rt.data(), rt.size() * 8, hipMemcpyHostToDevice, s), "upload rho_t"));
  VEMB_TRY(hip_rc(hipMemcpyAsync(p->a.rho, rt.data(), rt.size() * 8, hipMemcpyHostToDevice, s), "upload rho"));
  VEMB_TRY(hip_rc(hipMemsetAsync(p->a.Lam, 0, (size_t)P * n * n * 8, s), "zero Lam"));
  VEMB_TRY(hip_rc(hipMemsetAsync(p->a.Lam1, 0, (size_t)P * m * m * 8, s), "zero Lam1"));
  VEMB_TRY(hip_rc(hipMemsetAsync(p->a.Lam2, 0, (size_t)P * m * m * 8, s), "zero Lam2"));
  VEMB_TRY(hip_rc(hipStreamSynchronize(s), "initial upload"));
  p->t = 0;
  return VEMB_OK;
}

hipEvent_t take_event(vemb_problem* p) {
  if (!p->free_events.empty()) {
    hipEvent_t e = p->free_events.back();
    p->free_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Runs one launcher, bracketed by events when profiling is on.
template <typename F>
int timed(vemb_problem* p, int id, const char* what, F&& launch, hipStream_t st = nullptr) {
  if (!st) st = p->stream;
  hipEvent_t a = nullptr, b = nullptr;
  const bool on = p->profiling && ((p->prof_mask >> id) & 1u) && p->t % p->prof_every == 0;
  if (on) {
    a = take_event(p);
    b = take_event(p);
    if (a) hipEventRecord(a, st);
  }
  int rc = hip_rc(launch(), what);
  if (on && a && b) {
    hipEventRecord(b, st);
    p->marks.push_back({id, a, b});
  }
  return rc;
}

int drain_marks(vemb_problem* p) {
  if (p->marks.empty()) return VEMB_OK;
  VEMB_TRY(hip_rc(hipStreamSynchronize(p->stream), "profile sync"));
  for (auto& mk : p->marks) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, mk.start, mk.stop) == hipSuccess) {
      p->prof_ms[mk.id] += ms;
      p->prof_n[mk.id] += 1;
    }
    p->free_events.push_back(mk.start);
    p->free_events.push_back(mk.stop);
  }
  p->marks.clear();
  return VEMB_OK;
}

// ---------------------------------------------------------------------------
// Autotuner: threads per workgroup of the LDS Jacobi solver (256 / 512 / 1024),
// chosen per (device, n, real/complex, precision, batch size rounded up to a
// power of two) by timing the candidates with HIP events on seeded synthetic
// matrices shaped like ADMM iterates.  Results are cached in memory and in a
// text file: $VEMB_TUNE_CACHE, default $HOME/.cache/vemb_tune.txt ("none"
// keeps the cache in memory only).
// ---------------------------------------------------------------------------
std::mutex g_tune_mu;
std::map<std::string, int> g_tune;
bool g_tune_loaded = false;

std::string tune_path() {
  const char* env = std::getenv("VEMB_TUNE_CACHE");
  if (env) return std::string(env) == "none" ? std::string() : std::string(env);
  const char* home = std::getenv("HOME");
  return home ? std::string(home) + "/.cache/vemb_tune.txt" : std::string();
}

void tune_load() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const std::string path = tune_path();
  if (path.empty()) return;
  if (FILE* f = std::fopen(path.c_str(), "r")) {
    char key[256];
    int v = 0;
    while (std::fscanf(f, "%255s %d", key, &v) == 2) g_tune[key] = v;
    std::fclose(f);
  }
}

void tune_store(const std::string& key, int v) {
  g_tune[key] = v;
  const std::string path = tune_path();
  if (path.empty()) return;
  const size_t slash = path.rfind('/');
  if (slash != std::string::npos && slash > 0) {
    // create the directory if missing; no shell is spawned
    std::error_code ec;
    std::filesystem::create_directories(path.substr(0, slash), ec);
    if (ec) {
      std::fprintf(stderr, "vemb: autotuner cache directory for %s: %s (result kept in memory)\n", path.c_str(),
                   ec.message().c_str());
      return;
    }
  }
  if (FILE* f = std::fopen(path.c_str(), "a")) {
    std::fprintf(f, "%s %d\n", key.c_str(), v);
    std::fclose(f);
  } else {
    std::fprintf(stderr, "vemb: cannot append to the autotuner cache %s (result kept in memory)\n", path.c_str());
  }
}

// Seeded symmetric / Hermitian test matrices: diagonal ~ U[0, 2/n], off-diagonal ~ U[-1, 1]/(2n),
// roughly half of the eigenvalues negative, like rho - Lambda/mu.
void synth_batch(std::vector<double>& h, int n, int count, bool cplx) {
  const int w = cplx ? 2 : 1;
  h.assign((size_t)count * n * n * w, 0.0);
  uint64_t x = 0x9E3779B97F4A7C15ull ^ ((uint64_t)n << 32) ^ (uint64_t)count;
  auto next = [&]() {  // xorshift64*
    x ^= x >> 12;
    x ^= x << 25;
    x ^= x >> 27;
    return (double)((x * 0x2545F4914F6CDD1Dull) >> 11) * (1.0 / 9007199254740992.0);
  };
  for (int b = 0; b < count; ++b)
    for (int i = 0; i < n; ++i)
      for (int j = i; j < n; ++j) {
        double re = (i == j) ? 2.0 * next() / n - 0.5 / n : (2.0 * next() - 1.0) / (2.0 * n);
        double im = (cplx && i != j) ? (2.0 * next() - 1.0) / (2.0 * n) : 0.0;
        const size_t o1 = ((size_t)b * n * n + (size_t)i * n + j) * w, o2 = ((size_t)b * n * n + (size_t)j * n + i) * w;
        h[o1] = re;
        h[o2] = re;
        if (cplx) {
          h[o1 + 1] = im;
          h[o2 + 1] = -im;
        }
      }
}

}  // namespace

int vemb::tuned_tpb(int n, bool cplx, int precision, int count, hipStream_t st) {
  const int np = (n + 1) & ~1;
  if (np < 16 || np > 64 || count <= 0) return 256;  // one variant only
  int bucket = 1;
  while (bucket < count) bucket <<= 1;
  bucket = std::min(bucket, 4096);
  int dev = 0;
  hipGetDevice(&dev);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return 256;
  char key[256];
  std::snprintf(key, sizeof(key), "v3:%s:cu%d:n%d:%s:p%d:b%d", prop.gcnArchName, prop.multiProcessorCount, n,
                cplx ? "c" : "r", precision, bucket);
  std::lock_guard<std::mutex> lock(g_tune_mu);
  tune_load();
  auto it = g_tune.find(key);
  if (it != g_tune.end()) return it->second;
  std::vector<double> h;
  synth_batch(h, n, bucket, cplx);
  // the iteration's solves are warm-started from the previous eigenvectors: time a warm
  // solve of a slightly moved batch (relative change 1e-3) after a cold solve of the first
  std::vector<double> h2(h);
  {
    std::vector<double> pert;
    synth_batch(pert, n, bucket, cplx);
    for (size_t i = 0; i < h2.size(); ++i) h2[i] += 1e-3 * pert[(i * 7919) % pert.size()];
    const int w = cplx ? 2 : 1;  // keep the moved batch symmetric / Hermitian
    for (int b = 0; b < bucket; ++b)
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < i; ++j)
          for (int c = 0; c < w; ++c) {
            const size_t lo = (((size_t)b * n + i) * n + j) * w + c, up = (((size_t)b * n + j) * n + i) * w + c;
            h2[lo] = c == 0 ? h2[up] : -h2[up];
          }
  }
  const size_t bytes = h.size() * sizeof(double);
  DeviceMemory mem;
  double* din = static_cast<double*>(mem.get(bytes));
  double* din2 = static_cast<double*>(mem.get(bytes));
  double* dout = static_cast<double*>(mem.get(bytes));
  double* dv = static_cast<double*>(mem.get(bytes));
  int best = 256;
  if (din && din2 && dout && dv &&
      hipMemcpyAsync(din, h.data(), bytes, hipMemcpyHostToDevice, st) == hipSuccess &&
      hipMemcpyAsync(din2, h2.data(), bytes, hipMemcpyHostToDevice, st) == hipSuccess) {
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    float best_ms = 1e30f;
    std::vector<int> cand = {256, 512, 1024};
    if (n == 64) cand.insert(cand.begin(), {kTpbRegister8, kTpbRegister4});
    for (int tpb : cand) {
      float t_min = 1e30f;
      bool ok = true;
      for (int rep = 0; rep < 3 && ok; ++rep) {
        ok = launch_psd_batched(din, dout, n, bucket, cplx, precision, 40, nullptr, dv, tpb, st, 1) == hipSuccess;
        hipEventRecord(e0, st);
        ok = ok && launch_psd_batched(din2, dout, n, bucket, cplx, precision, 40, nullptr, dv, tpb, st, 0) ==
                       hipSuccess;
        hipEventRecord(e1, st);
        hipEventSynchronize(e1);
        float ms = 0.f;
        hipEventElapsedTime(&ms, e0, e1);
        if (rep > 0) t_min = std::min(t_min, ms);  // first launch warms up
      }
      if (ok && t_min < best_ms) {
        best_ms = t_min;
        best = tpb;
      }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
  }
  hipStreamSynchronize(st);
  mem.release();
  hipGetLastError();  // a failed candidate must not leak its error into the caller
  tune_store(key, best);
  return best;
}

namespace {

bool all_finite(const double* v, size_t count) {
  for (size_t i = 0; i < count; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

// Penalties, step and the coefficients of the pair update's closed-form inverse (eq. rhoijUpdate):
// rho = a R + (b/m)(Tr_2 R x I + I x Tr_1 R) + (c/m^2) Tr R I.
void set_parameters(StepArgs& a, double mu, double nu, double eps) {
  const int m = a.m;
  a.mu = mu;
  a.nu = nu;
  a.eps = eps;
  a.a = 1.0 / mu;
  a.b = 1.0 / (mu + nu * m) - 1.0 / mu;
  a.c = 1.0 / (mu + 2 * nu * m) - 2.0 / (mu + nu * m) + 1.0 / mu;
}

}  // namespace

extern "C" {

const char* vemb_last_error(void) { return g_last_error.c_str(); }

int vemb_set_allocator(vemb_alloc_fn alloc_fn, vemb_free_fn free_fn, void* ctx) {
  if ((alloc_fn == nullptr) != (free_fn == nullptr))
    return fail(VEMB_E_INVALID, "vemb_set_allocator needs both functions, or neither");
  std::lock_guard<std::mutex> lock(g_alloc_mu);
  if (g_live_objects > 0)
    return fail(VEMB_E_INVALID, std::to_string(g_live_objects) + " library objects are alive: destroy them before "
                                "switching allocators");
  g_alloc.alloc = alloc_fn;
  g_alloc.free = free_fn;
  g_alloc.ctx = alloc_fn ? ctx : nullptr;
  return VEMB_OK;
}

int vemb_create_problem(const vemb_hamiltonian* H, const vemb_lattice* lat, const vemb_clusters* cl,
                        const vemb_options* opts, void* hip_stream, vemb_problem** out) {
  if (!H || !lat || !cl || !out || (H->nterms > 0 && !H->terms)) return fail(VEMB_E_INVALID, "NULL argument");
  *out = nullptr;
  vemb_options o;
  Geometry g{};
  std::string perr;
  int prc = normalize_options(opts, o, perr);
  if (prc == VEMB_OK) prc = parse_geometry(*lat, *cl, g, perr);
  if (prc != VEMB_OK) return fail(prc, perr);
  const int n_op = o.opset == VEMB_OPSET_COMPLETE ? g.n : 3 * g.L;
  // eigensolver capacity: pair blocks n x n (real), momentum blocks n_op x n_op (complex), n <= 256
  if (g.n > 256 || n_op > 256) return fail(VEMB_E_UNSUPPORTED, "matrices above 256 x 256 are not supported");

  auto* p = new vemb_problem();
  object_created();
  p->g = g;
  p->P = g.M - 1;
  p->n_op = n_op;
  p->opt = o;
  p->stream = static_cast<hipStream_t>(hip_stream);
  std::string err;
  int rc = build_model(*H, g, p->host, err, o.fermionic != 0);
  if (rc != VEMB_OK) {
    delete p;  // nothing on the device yet
    object_destroyed();
    return fail(rc, err);
  }
  std::vector<double> tw, wk;
  build_momenta(g, tw, wk, p->Ku);
  if (o.opset == VEMB_OPSET_PAULI1) build_pauli1_tables(g.L, p->ops_host);

  const int m = g.m, n = g.n, M = g.M, P = p->P, k = n_op, Ku = p->Ku;
  StepArgs& a = p->a;
  a.M = M;
  a.P = P;
  a.m = m;
  a.n = n;
  a.n_op = k;
  a.Ku = Ku;
  a.opset = o.opset;
  a.fermionic = o.fermionic;
  a.sign = o.sign < 0 ? -1.0 : 1.0;
  a.active = 1;
  set_parameters(a, o.mu, o.nu, o.eps);
  auto cleanup = [&](int code) {
    vemb_destroy(p);
    return code;
  };
  if (hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&p->fork_ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&p->join_ev, hipEventDisableTiming) != hipSuccess)
    return cleanup(fail(VEMB_E_HIP, "side stream / events"));
  const size_t nh = p->host.Hd.size() / ((size_t)n * n);
  if ((rc = dalloc(p, &p->H0, (size_t)m * m)) || (rc = dalloc(p, &p->Hd, nh * n * n)) ||
      (rc = dalloc(p, &p->hd_index, (size_t)P)) || (rc = dalloc(p, &p->tw, tw.size())) ||
      (rc = dalloc(p, &p->wk, wk.size())) || (rc = dalloc(p, &p->ops, 1)) ||
      (rc = dalloc(p, &a.X, (size_t)M * k * k)) || (rc = dalloc(p, &a.Xp, (size_t)M * k * k)) ||
      (rc = dalloc(p, &a.Xh, (size_t)2 * Ku * k * k)) || (rc = dalloc(p, &a.rho0, (size_t)m * m)) ||
      (rc = dalloc(p, &a.rho, (size_t)P * n * n)) || (rc = dalloc(p, &a.rho_t, (size_t)P * n * n)) ||
      (rc = dalloc(p, &a.Lam, (size_t)P * n * n)) || (rc = dalloc(p, &a.Lam1, (size_t)P * m * m)) ||
      (rc = dalloc(p, &a.Lam2, (size_t)P * m * m)) || (rc = dalloc(p, &a.tr2, (size_t)P * m * m)) ||
      (rc = dalloc(p, &a.tr1, (size_t)P * m * m)) || (rc = dalloc(p, &a.e_pair, (size_t)P)) ||
      (rc = dalloc(p, &a.feas, (size_t)P)) || (rc = dalloc(p, &a.scal, 4)) ||
      (rc = dalloc(p, &a.Kbuf, (size_t)P * n * n + (size_t)m * m)) || (rc = dalloc(p, &a.lmin, (size_t)P + 1)) ||
      (n <= 128 && (rc = dalloc(p, &p->Kv, (size_t)P * n * n))) ||
      (rc = dalloc(p, &a.sweeps, (size_t)(2 * P + Ku + 1))) ||
      (rc = dalloc(p, &a.Vpair, (size_t)P * n * n)) || (rc = dalloc(p, &a.Vmom, (size_t)2 * Ku * k * k)) ||
      (n > 64 && ((rc = dalloc(p, (double**)&a.wscr_pair, (size_t)P * n * n)) ||
                  (rc = dalloc(p, (double**)&a.tscr_pair, (size_t)P * n * n)))) ||
      (n > 64 && (rc = dalloc(p, (char**)&p->sign_pair, sign_work_bytes(n, P, false)))) ||
      (n > 128 && ((rc = dalloc(p, &p->slice_x, (size_t)P * n)) || (rc = dalloc(p, &p->slice_sigma, (size_t)P)) ||
                   (rc = dalloc(p, &p->slice_flags, (size_t)P)) || (rc = dalloc(p, &p->slice_nflag, 1)))) ||
      (k > 64 && (rc = dalloc(p, (char**)&p->sign_mom, sign_work_bytes(k, Ku, true)))) ||
      (k > 64 && ((rc = dalloc(p, (double**)&a.wscr_mom, (size_t)2 * Ku * k * k)) ||
                  (rc = dalloc(p, (double**)&a.tscr_mom, (size_t)2 * Ku * k * k)))))
    return cleanup(rc);
  hipStream_t s = p->stream;
  if ((rc = hip_rc(hipMemcpyAsync(p->H0, p->host.H0.data(), (size_t)m * m * 8, hipMemcpyHostToDevice, s), "upload H0")) ||
      (nh && (rc = hip_rc(hipMemcpyAsync(p->Hd, p->host.Hd.data(), p->host.Hd.size() * 8, hipMemcpyHostToDevice, s), "upload Hd"))) ||
      (rc = hip_rc(hipMemcpyAsync(p->hd_index, p->host.hd_index.data(), (size_t)P * sizeof(int), hipMemcpyHostToDevice, s), "upload index")) ||
      (rc = hip_rc(hipMemcpyAsync(p->tw, tw.data(), tw.size() * 8, hipMemcpyHostToDevice, s), "upload twiddles")) ||
      (rc = hip_rc(hipMemcpyAsync(p->wk, wk.data(), wk.size() * 8, hipMemcpyHostToDevice, s), "upload weights")) ||
      (rc = hip_rc(hipMemcpyAsync(p->ops, &p->ops_host, sizeof(OpTables), hipMemcpyHostToDevice, s), "upload ops")) ||
      (rc = hip_rc(hipMemsetAsync(a.sweeps, 0, sizeof(int) * (2 * P + Ku + 1), s), "zero sweeps")) ||
      (rc = hip_rc(hipMemsetAsync(a.e_pair, 0, sizeof(double) * P, s), "zero e_pair")) ||
      (rc = hip_rc(hipMemsetAsync(a.feas, 0, sizeof(double) * P, s), "zero feas")) ||
      (rc = hip_rc(hipMemsetAsync(a.scal, 0, sizeof(double) * 4, s), "zero scal")) ||
      (p->slice_x && (rc = hip_rc(hipMemsetAsync(p->slice_x, 0, sizeof(double) * P * n, s), "zero slice vectors"))))
    return cleanup(rc);
  a.H0 = p->H0;
  a.Hd = p->Hd;
  a.hd_index = p->hd_index;
  a.tw = p->tw;
  a.wk = p->wk;
  a.ops = p->ops;
  if ((rc = upload_initial_state(p))) return cleanup(rc);
  if (o.tpb == kTpbRegister8 || o.tpb == kTpbRegister4 || o.tpb == 256 || o.tpb == 512 || o.tpb == 1024) {
    p->tpb_pair = p->tpb_mom = o.tpb;
  } else {
    p->tpb_pair = tuned_tpb(n, false, solve_precision(o.precision), P, s);
    p->tpb_mom = tuned_tpb(k, true, solve_precision(o.precision), Ku, s);
  }
  *out = p;
  return VEMB_OK;
}

int vemb_problem_info(const vemb_problem* p, vemb_info* info) {
  if (!p || !info) return fail(VEMB_E_INVALID, "NULL argument");
  info->M = p->g.M;
  info->P = p->P;
  info->L = p->g.L;
  info->m = p->g.m;
  info->n = p->g.n;
  info->n_op = p->n_op;
  info->Mx = p->g.Mx;
  info->My = p->g.My;
  info->K_unique = p->Ku;
  info->t = p->t;
  return VEMB_OK;
}

namespace {
// Iterations with pair and momentum blocks of 33..64 that the autotuner gave the same LDS solver variant
// run both projections in one launch.
bool fused_projections(const vemb_problem* p) {
  return !p->sign_pair && !p->sign_mom && fused_projection_fits(p->a.n, p->a.n_op) &&
         p->tpb_pair == kFusedThreads && p->tpb_mom == kFusedThreads;
}

int diag_enqueue(vemb_problem* p);
int diag_collect(vemb_problem* p, double* lb, double* e, double* f);

// The watchdog of vemb_options.lb_every, after iteration t: read back the diagnostics queued one
// interval ago, apply vemb_divergence_check to the feasibility history, queue the current ones.
int watchdog(vemb_problem* p) {
  if (p->diag_pending) {
    double lb = 0.0, e = 0.0, f = 0.0;
    const int rc = diag_collect(p, &lb, &e, &f);
    p->feas_hist.push_back(f);
    const int w = vemb_divergence_check(p->feas_hist.data(), (int)p->feas_hist.size(), lb, e);
    if (rc != VEMB_OK || w != VEMB_OK) {
      const int code = w != VEMB_OK ? w : rc;
      return fail(code, "watchdog at iteration " + std::to_string(p->t - p->opt.lb_every) + ": " +
                            std::string(vemb_last_error()));
    }
  }
  return diag_enqueue(p);
}

// prec: VEMB_FP64, or the problem's MIXED / FP32 mode, whose eigensolves run in FP32 (sweeps, rebuild and
// sign-function products; state and diagnostics stay FP64).
// Adaptive parameters (vemb_options.adapt_every), after iteration t: the FP64 diagnostics (feasErr of eq.
// feasErr and the relative primal-dual gap |E_p - LB| / |LB|), then one decision of the joint scale of
// (mu, nu, eps): grown when both fell by more than a relative dead band, shrunk when either rose by more
// (a quantity whose two values both lie at the rounding floor counts as neither).  Synchronises the stream.
constexpr double kAdaptGrow = 1.25, kAdaptShrink = 0.5, kAdaptMax = 8.0, kAdaptDead = 1e-6, kAdaptFloor = 1e-12;

int trend(double x, double x_prev) {
  if (x <= kAdaptFloor && x_prev <= kAdaptFloor) return 0;
  if (x < x_prev * (1.0 - kAdaptDead)) return -1;
  if (x > x_prev * (1.0 + kAdaptDead)) return 1;
  return 0;
}

double next_scale(double c, double f, double g, double f_prev, double g_prev) {
  const int tf = trend(f, f_prev), tg = trend(g, g_prev);
  if (tf > 0 || tg > 0)
    c *= kAdaptShrink;
  else if (tf < 0 && tg < 0)
    c *= kAdaptGrow;
  return std::min(std::max(c, 1.0), kAdaptMax);
}

int adapt_check(vemb_problem* p) {
  double lb = 0.0, e = 0.0, f = 0.0;
  VEMB_TRY(vemb_diagnostics(p, &lb, &e, &f));
  const double g = std::fabs(e - lb) / std::fabs(lb);
  if (!std::isfinite(g)) return fail(VEMB_E_NUMERIC, "non-finite gap at iteration " + std::to_string(p->t));
  if (p->adapt_last >= 0.0) {
    p->adapt_scale = next_scale(p->adapt_scale, f, g, p->adapt_last, p->adapt_last_gap);
    const double c = p->adapt_scale;
    set_parameters(p->a, c * p->opt.mu, c * p->opt.nu, c * p->opt.eps);
  }
  p->adapt_last = f;
  p->adapt_last_gap = g;
  return VEMB_OK;
}

int run_iterations(vemb_problem* p, int iters, int prec) {
  const StepArgs& a = p->a;
  hipStream_t s = p->stream;
  const int ms = p->opt.max_sweeps;
  const int sp = solve_precision(prec);
  for (int it = 0; it < iters; ++it) {
    const int refresh = p->opt.warm_refresh;
    int cold = (!p->v_valid || refresh < 0 || p->t % refresh == 0) ? 1 : 0;
    // FP64 solves warm-started from FP32 eigenvectors restore their orthonormality first
    if (!cold && sp == VEMB_FP64 && p->v_fp32) cold = 2;
    VEMB_TRY(timed(p, VEMB_K_PAIR_UPDATE, "pair update", [&] { return launch_pair_update(a, s); }));
    VEMB_TRY(timed(p, VEMB_K_PAIR_XSTEP, "pair X step", [&] { return launch_pair_xstep(a, s); }));
    if (fused_projections(p)) {
      // both projections in one launch after the forward DFT: one stream, no fork and join
      VEMB_TRY(timed(p, VEMB_K_CLUSTER, "cluster update", [&] { return launch_cluster_update(a, s); }));
      VEMB_TRY(timed(p, VEMB_K_DFT_FWD, "forward DFT", [&] { return launch_dft_forward(a, s); }));
      VEMB_TRY(timed(p, VEMB_K_PROJ, "projections", [&] {
        return launch_projections_fused(a.rho, a.Lam, a.rho_t, a.feas, a.n, a.P, a.mu, a.Xh, a.n_op, a.Ku, ms,
                                        a.sweeps, a.Vpair, a.Vmom, cold, s, sp);
      }));
      VEMB_TRY(timed(p, VEMB_K_DFT_INV, "inverse DFT", [&] { return launch_dft_inverse(a, s); }));
      p->v_valid = true;
      p->v_fp32 = sp != VEMB_FP64;
      ++p->t;
      if (p->opt.lb_every > 0 && p->t % p->opt.lb_every == 0) VEMB_TRY(watchdog(p));
      if (p->opt.adapt_every > 0 && p->t % p->opt.adapt_every == 0) VEMB_TRY(adapt_check(p));
      continue;
    }
    // fork: pair projection on the side stream (reads rho, Lambda; writes rho_t,
    // Lambda, feas, Vpair -- nothing the main branch touches)
    hipStream_t s2 = p->side;
    VEMB_TRY(hip_rc(hipEventRecord(p->fork_ev, s), "fork"));
    VEMB_TRY(hip_rc(hipStreamWaitEvent(s2, p->fork_ev, 0), "fork"));
    VEMB_TRY(timed(p, VEMB_K_PAIR_PROJ, "pair projection", [&] {
      if (p->sign_pair)
        return launch_pair_projection_sign(a.rho, a.Lam, a.rho_t, a.feas, a.n, a.P, a.mu, a.sweeps, p->sign_pair,
                                           s2, sp);
      return launch_pair_projection(a.rho, a.Lam, a.rho_t, a.feas, a.n, a.P, a.mu, sp, ms, a.sweeps, a.Vpair, cold,
                                    p->tpb_pair, s2);
    }, s2));
    VEMB_TRY(hip_rc(hipEventRecord(p->join_ev, s2), "join"));
    VEMB_TRY(timed(p, VEMB_K_CLUSTER, "cluster update", [&] { return launch_cluster_update(a, s); }));
    VEMB_TRY(timed(p, VEMB_K_DFT_FWD, "forward DFT", [&] { return launch_dft_forward(a, s); }));
    VEMB_TRY(timed(p, VEMB_K_MOM_PROJ, "momentum projection", [&] {
      if (p->sign_mom) return launch_momentum_projection_sign(a.Xh, a.n_op, a.Ku, a.sweeps + a.P, p->sign_mom, s, sp);
      return launch_momentum_projection(a.Xh, a.n_op, a.Ku, sp, ms, a.sweeps + a.P, a.Vmom, cold, p->tpb_mom, s);
    }));
    VEMB_TRY(timed(p, VEMB_K_DFT_INV, "inverse DFT", [&] { return launch_dft_inverse(a, s); }));
    VEMB_TRY(hip_rc(hipStreamWaitEvent(s, p->join_ev, 0), "join"));
    p->v_valid = true;
    p->v_fp32 = sp != VEMB_FP64;
    ++p->t;
    if (p->opt.lb_every > 0 && p->t % p->opt.lb_every == 0) VEMB_TRY(watchdog(p));
    if (p->opt.adapt_every > 0 && p->t % p->opt.adapt_every == 0) VEMB_TRY(adapt_check(p));
  }
  return VEMB_OK;
}
}  // namespace

namespace {
// X <- Pi(X') through the momentum blocks (steps 7-9 alone), FP64, cold eigensolves.
int project_x(vemb_problem* p) {
  const StepArgs& a = p->a;
  hipStream_t s = p->stream;
  const int ms = p->opt.max_sweeps;
  VEMB_TRY(hip_rc(launch_dft_forward(a, s), "forward DFT"));
  if (p->sign_mom)
    VEMB_TRY(hip_rc(launch_momentum_projection_sign(a.Xh, a.n_op, a.Ku, a.sweeps + a.P, p->sign_mom, s, VEMB_FP64),
                    "momentum projection"));
  else if (a.n_op > 64)
    VEMB_TRY(hip_rc(launch_momentum_projection_big(a.Xh, a.n_op, a.Ku, VEMB_FP64, ms, a.sweeps + a.P, a.Vmom, 1,
                                                   a.wscr_mom, a.tscr_mom, s),
                    "momentum projection"));
  else
    VEMB_TRY(hip_rc(launch_momentum_projection(a.Xh, a.n_op, a.Ku, VEMB_FP64, ms, a.sweeps + a.P, a.Vmom, 1,
                                               p->tpb_mom, s),
                    "momentum projection"));
  return hip_rc(launch_dft_inverse(a, s), "inverse DFT");
}

int check_ring(const vemb_problem* p) {
  if (p->g.My != 1) return fail(VEMB_E_UNSUPPORTED, "the warm-start encoding covers rings (one-dimensional cluster lattices)");
  return VEMB_OK;
}
}  // namespace

int vemb_warm_size(const vemb_problem* p, int near, int64_t* count) {
  if (!p || !count || near < 1) return fail(VEMB_E_INVALID, "bad arguments to vemb_warm_size");
  VEMB_TRY(check_ring(p));
  *count = warm_layout(p->a, near).total;
  return VEMB_OK;
}

int vemb_warm_encode(vemb_problem* p, int near, float* vec) {
  if (!p || !vec || near < 1) return fail(VEMB_E_INVALID, "bad arguments to vemb_warm_encode");
  VEMB_TRY(check_ring(p));
  if (p->g.M < near + 1) return fail(VEMB_E_UNSUPPORTED, "encoding needs more clusters than near distances");
  return hip_rc(launch_warm_encode(p->a, near, vec, p->stream), "warm-start encode");
}

int vemb_warm_start(vemb_problem* p, int near, const float* vec) { return vemb_warm_start_ex(p, near, vec, 0); }

int vemb_warm_start_ex(vemb_problem* p, int near, const float* vec, int far_cold) {
  if (!p || !vec || near < 1) return fail(VEMB_E_INVALID, "bad arguments to vemb_warm_start");
  VEMB_TRY(check_ring(p));
  VEMB_TRY(hip_rc(launch_warm_decode(p->a, near, vec, p->stream, far_cold), "warm-start decode"));
  VEMB_TRY(project_x(p));
  p->t = 0;
  p->v_valid = false;
  p->k_valid = false;
  return VEMB_OK;
}

int vemb_step(vemb_problem* p, int iters) {
  if (!p || iters < 0) return fail(VEMB_E_INVALID, "bad arguments to vemb_step");
  return run_iterations(p, iters, p->opt.precision);
}

int vemb_refine(vemb_problem* p, int iters) {
  if (!p || iters < 0) return fail(VEMB_E_INVALID, "bad arguments to vemb_refine");
  return run_iterations(p, iters, VEMB_FP64);
}

int vemb_primal_energy(vemb_problem* p, double* e_per_site, double* feas_err) {
  if (!p) return fail(VEMB_E_INVALID, "NULL problem");
  const int P = p->P;
  std::vector<double> ep(P), fe(P), sc(4);
  hipStream_t s = p->stream;
  VEMB_TRY(hip_rc(hipMemcpyAsync(ep.data(), p->a.e_pair, P * 8, hipMemcpyDeviceToHost, s), "copy energies"));
  VEMB_TRY(hip_rc(hipMemcpyAsync(fe.data(), p->a.feas, P * 8, hipMemcpyDeviceToHost, s), "copy feas"));
  VEMB_TRY(hip_rc(hipMemcpyAsync(sc.data(), p->a.scal, 4 * 8, hipMemcpyDeviceToHost, s), "copy scalars"));
  VEMB_TRY(hip_rc(hipStreamSynchronize(s), "primal energy sync"));
  double e = sc[0], f = sc[1];
  for (int d = 0; d < P; ++d) {
    e += 0.5 * ep[d];
    f += fe[d];
  }
  if (e_per_site) *e_per_site = e / p->g.L;
  if (feas_err) *feas_err = std::sqrt(f / (p->g.M - 1));
  if (!std::isfinite(e) || !std::isfinite(f)) return fail(VEMB_E_NUMERIC, "non-finite energy or feasibility");
  return VEMB_OK;
}

namespace {
// Bound matrices and their smallest eigenvalues (enqueued); the pair solves start from the
// eigenvectors of the previous bound evaluation.
int enqueue_bound(vemb_problem* p) {
  const StepArgs& a = p->a;
  hipStream_t s = p->stream;
  const int P = p->P, n = a.n, m = a.m;
  VEMB_TRY(timed(p, VEMB_K_BOUND_BUILD, "bound build", [&] { return launch_bound_build(a, s); }));
  VEMB_TRY(timed(p, VEMB_K_LMIN, "pair lambda_min", [&] {
    if (n > 128) {
      // spectral slicing, in FP64 in every precision mode (an FP32 sign function leaves ~1e-5 of other
      // eigenvectors in the Ritz space, ~1e-9 in the value); the first evaluation (no Ritz vectors yet)
      // takes two passes up front
      const int passes = p->slice_started ? 1 : 2;
      p->slice_started = true;
      hipError_t e = hipSuccess;
      for (int k = 0; k < passes && e == hipSuccess; ++k)
        e = launch_lambda_min_slice(a.Kbuf, p->slice_x, p->slice_sigma, a.lmin, p->slice_flags, p->slice_nflag, n, P,
                                    p->sign_pair, s, VEMB_FP64);
      return e;
    }
    const int cold = (!p->k_valid || p->k_uses % 16 == 0) ? 1 : 0;
    return launch_lambda_min(a.Kbuf, a.lmin, n, P, p->opt.max_sweeps, a.sweeps + P + a.Ku, s, p->tpb_pair, p->Kv,
                             cold);
  }));
  if (n <= 128 && p->Kv) {
    p->k_valid = true;
    ++p->k_uses;
  }
  return timed(p, VEMB_K_LMIN, "cluster lambda_min", [&] {
    return launch_lambda_min(a.Kbuf + (size_t)P * n * n, a.lmin + P, m, 1, p->opt.max_sweeps, nullptr, s);
  });
}

constexpr int kSlicePasses = 4;

// After a synchronised bound evaluation with matrices above 128: blocks whose slicing pass was flagged
// (more eigenvalues below the shift than the Ritz space can hold) get further passes, each starting from
// its latest Ritz vector, then the streamed Jacobi solve if any is still flagged; lm (host, P values) is
// refreshed when anything ran.  Later work already queued on the stream runs first (the bound buffers are
// only rewritten by the next evaluation).
int slice_fixup(vemb_problem* p, double* lm) {
  const StepArgs& a = p->a;
  if (a.n <= 128) return VEMB_OK;
  hipStream_t s = p->stream;
  int nf = 0;
  auto read_flags = [&] {
    VEMB_TRY(hip_rc(hipMemcpyAsync(&nf, p->slice_nflag, sizeof(int), hipMemcpyDeviceToHost, s), "copy slice flags"));
    return hip_rc(hipStreamSynchronize(s), "slice flags sync");
  };
  VEMB_TRY(read_flags());
  if (!nf) return VEMB_OK;
  for (int pass = 1; pass < kSlicePasses && nf; ++pass) {
    VEMB_TRY(hip_rc(launch_lambda_min_slice(a.Kbuf, p->slice_x, p->slice_sigma, a.lmin, p->slice_flags,
                                            p->slice_nflag, a.n, p->P, p->sign_pair, s, VEMB_FP64),
                    "slicing pass"));
    VEMB_TRY(read_flags());
  }
  if (nf)
    VEMB_TRY(hip_rc(launch_eigvals_big(a.Kbuf, nullptr, a.lmin, a.n, p->P, false, p->opt.max_sweeps,
                                       a.sweeps + p->P + a.Ku, a.wscr_pair, a.tscr_pair, s),
                    "pair lambda_min (streamed)"));
  VEMB_TRY(hip_rc(hipMemcpyAsync(lm, a.lmin, (size_t)p->P * 8, hipMemcpyDeviceToHost, s), "copy lambda_min"));
  return hip_rc(hipStreamSynchronize(s), "lambda_min sync");
}

double bound_from(const vemb_problem* p, const std::vector<double>& lm) {
  const int P = p->P;
  double sum = 0.0;
  for (int d = 0; d < P; ++d) sum += lm[d];
  return (lm[P] + 0.5 * sum) / p->g.L;
}
}  // namespace

int vemb_dual_bound(vemb_problem* p, double* lb) {
  if (!p || !lb) return fail(VEMB_E_INVALID, "NULL argument");
  VEMB_TRY(enqueue_bound(p));
  std::vector<double> lm(p->P + 1);
  VEMB_TRY(hip_rc(hipMemcpyAsync(lm.data(), p->a.lmin, (p->P + 1) * 8, hipMemcpyDeviceToHost, p->stream),
                  "copy lambda_min"));
  VEMB_TRY(hip_rc(hipStreamSynchronize(p->stream), "dual bound sync"));
  VEMB_TRY(slice_fixup(p, lm.data()));
  VEMB_TRY(drain_marks(p));  // the stream is idle: recycle the timing events now
  *lb = bound_from(p, lm);
  if (!std::isfinite(*lb)) return fail(VEMB_E_NUMERIC, "non-finite lower bound");
  return VEMB_OK;
}

int vemb_diagnostics(vemb_problem* p, double* lb, double* e_per_site, double* feas_err) {
  if (!p || !lb) return fail(VEMB_E_INVALID, "NULL argument");
  const int P = p->P;
  hipStream_t s = p->stream;
  std::vector<double> ep(P), fe(P), sc(4), lm(P + 1);
  VEMB_TRY(hip_rc(hipMemcpyAsync(ep.data(), p->a.e_pair, P * 8, hipMemcpyDeviceToHost, s), "copy energies"));
  VEMB_TRY(hip_rc(hipMemcpyAsync(fe.data(), p->a.feas, P * 8, hipMemcpyDeviceToHost, s), "copy feas"));
  VEMB_TRY(hip_rc(hipMemcpyAsync(sc.data(), p->a.scal, 4 * 8, hipMemcpyDeviceToHost, s), "copy scalars"));
  VEMB_TRY(enqueue_bound(p));
  VEMB_TRY(hip_rc(hipMemcpyAsync(lm.data(), p->a.lmin, (P + 1) * 8, hipMemcpyDeviceToHost, s), "copy lambda_min"));
  VEMB_TRY(hip_rc(hipStreamSynchronize(s), "diagnostics sync"));
  VEMB_TRY(slice_fixup(p, lm.data()));
  VEMB_TRY(drain_marks(p));  // the stream is idle: recycle the timing events now
  *lb = bound_from(p, lm);
  double e = sc[0], f = sc[1];
  for (int d = 0; d < P; ++d) {
    e += 0.5 * ep[d];
    f += fe[d];
  }
  if (e_per_site) *e_per_site = e / p->g.L;
  if (feas_err) *feas_err = std::sqrt(f / (p->g.M - 1));
  if (!std::isfinite(*lb) || !std::isfinite(e) || !std::isfinite(f))
    return fail(VEMB_E_NUMERIC, "non-finite bound, energy or feasibility");
  return VEMB_OK;
}

namespace {
int diag_reduce(vemb_problem* p, const double* lm, const double* ep, const double* fe, const double* sc, double* lb,
                double* e_per_site, double* feas_err) {
  const int P = p->P;
  double sum = 0.0, e = sc[0], f = sc[1];
  for (int d = 0; d < P; ++d) {
    sum += lm[d];
    e += 0.5 * ep[d];
    f += fe[d];
  }
  *lb = (lm[P] + 0.5 * sum) / p->g.L;
  if (e_per_site) *e_per_site = e / p->g.L;
  if (feas_err) *feas_err = std::sqrt(f / (p->g.M - 1));
  if (!std::isfinite(*lb) || !std::isfinite(e) || !std::isfinite(f))
    return fail(VEMB_E_NUMERIC, "non-finite bound, energy or feasibility");
  return VEMB_OK;
}
}  // namespace

namespace {
int diag_enqueue(vemb_problem* p) {
  const int P = p->P;
  hipStream_t s = p->stream;
  if (!p->diag_host) {
    if (hipHostMalloc((void**)&p->diag_host, sizeof(double) * (3 * P + 5), hipHostMallocDefault) != hipSuccess) {
      p->diag_host = nullptr;
      return fail(VEMB_E_NOMEM, "pinned diagnostics buffer");
    }
    VEMB_TRY(hip_rc(hipEventCreateWithFlags(&p->diag_ev, hipEventDisableTiming), "diagnostics event"));
  }
  if (p->diag_pending) VEMB_TRY(hip_rc(hipEventSynchronize(p->diag_ev), "previous diagnostics"));
  double* h = p->diag_host;
  VEMB_TRY(hip_rc(hipMemcpyAsync(h + P + 1, p->a.e_pair, P * 8, hipMemcpyDeviceToHost, s), "copy energies"));
  VEMB_TRY(hip_rc(hipMemcpyAsync(h + 2 * P + 1, p->a.feas, P * 8, hipMemcpyDeviceToHost, s), "copy feas"));
  VEMB_TRY(hip_rc(hipMemcpyAsync(h + 3 * P + 1, p->a.scal, 4 * 8, hipMemcpyDeviceToHost, s), "copy scalars"));
  VEMB_TRY(enqueue_bound(p));
  VEMB_TRY(hip_rc(hipMemcpyAsync(h, p->a.lmin, (P + 1) * 8, hipMemcpyDeviceToHost, s), "copy lambda_min"));
  VEMB_TRY(hip_rc(hipEventRecord(p->diag_ev, s), "diagnostics event"));
  p->diag_pending = true;
  return VEMB_OK;
}

int diag_collect(vemb_problem* p, double* lb, double* e_per_site, double* feas_err) {
  VEMB_TRY(hip_rc(hipEventSynchronize(p->diag_ev), "diagnostics wait"));
  p->diag_pending = false;
  const int P = p->P;
  VEMB_TRY(slice_fixup(p, p->diag_host));
  const double* h = p->diag_host;
  return diag_reduce(p, h, h + P + 1, h + 2 * P + 1, h + 3 * P + 1, lb, e_per_site, feas_err);
}
}  // namespace

int vemb_diagnostics_enqueue(vemb_problem* p) {
  if (!p) return fail(VEMB_E_INVALID, "NULL problem");
  return diag_enqueue(p);
}

int vemb_diagnostics_collect(vemb_problem* p, double* lb, double* e_per_site, double* feas_err) {
  if (!p || !lb) return fail(VEMB_E_INVALID, "NULL argument");
  if (!p->diag_pending) return fail(VEMB_E_INVALID, "no diagnostics enqueued");
  return diag_collect(p, lb, e_per_site, feas_err);
}

int vemb_marginals(vemb_problem* p, int which, double* rho0, double* rho_pairs) {
  if (!p) return fail(VEMB_E_INVALID, "NULL problem");
  if (which != VEMB_RHO && which != VEMB_RHO_TILDE) return fail(VEMB_E_INVALID, "which must be RHO or RHO_TILDE");
  hipStream_t s = p->stream;
  const size_t m2 = (size_t)p->g.m * p->g.m, pn = (size_t)p->P * p->g.n * p->g.n;
  if (rho0) VEMB_TRY(hip_rc(hipMemcpyAsync(rho0, p->a.rho0, m2 * 8, hipMemcpyDeviceToHost, s), "copy rho0"));
  if (rho_pairs)
    VEMB_TRY(hip_rc(hipMemcpyAsync(rho_pairs, which == VEMB_RHO ? p->a.rho : p->a.rho_t, pn * 8,
                                   hipMemcpyDeviceToHost, s), "copy pairs"));
  return hip_rc(hipStreamSynchronize(s), "marginals sync");
}

int vemb_get_state(vemb_problem* p, vemb_state* st) {
  if (!p || !st) return fail(VEMB_E_INVALID, "NULL argument");
  hipStream_t s = p->stream;
  const size_t m2 = (size_t)p->g.m * p->g.m, n2 = (size_t)p->g.n * p->g.n, P = p->P;
  const size_t xk = (size_t)p->g.M * p->n_op * p->n_op;
  struct Item { double* host; const double* dev; size_t count; };
  const size_t vm = (size_t)2 * p->Ku * p->n_op * p->n_op;
  Item items[] = {{st->X, p->a.X, xk},           {st->rho0, p->a.rho0, m2},  {st->rho, p->a.rho, P * n2},
                  {st->rho_t, p->a.rho_t, P * n2}, {st->Lam, p->a.Lam, P * n2}, {st->Lam1, p->a.Lam1, P * m2},
                  {st->Lam2, p->a.Lam2, P * m2},   {st->Vpair, p->a.Vpair, P * n2}, {st->Vmom, p->a.Vmom, vm}};
  if ((st->Vpair || st->Vmom) && !p->v_valid)
    return fail(VEMB_E_INVALID, "get_state: no eigenvectors kept yet (run an iteration first)");
  for (const Item& it : items)
    if (it.host)
      VEMB_TRY(hip_rc(hipMemcpyAsync(it.host, it.dev, it.count * 8, hipMemcpyDeviceToHost, s), "get_state copy"));
  VEMB_TRY(hip_rc(hipStreamSynchronize(s), "get_state sync"));
  st->t = p->t;
  return VEMB_OK;
}

int vemb_set_state(vemb_problem* p, const vemb_state* st) {
  if (!p || !st) return fail(VEMB_E_INVALID, "NULL argument");
  const size_t m2 = (size_t)p->g.m * p->g.m, n2 = (size_t)p->g.n * p->g.n, P = p->P;
  const size_t xk = (size_t)p->g.M * p->n_op * p->n_op;
  struct Item { const double* host; double* dev; size_t count; };
  Item items[] = {{st->X, p->a.X, xk},           {st->rho0, p->a.rho0, m2},  {st->rho, p->a.rho, P * n2},
                  {st->rho_t, p->a.rho_t, P * n2}, {st->Lam, p->a.Lam, P * n2}, {st->Lam1, p->a.Lam1, P * m2},
                  {st->Lam2, p->a.Lam2, P * m2}};
  for (const Item& it : items) {
    if (!it.host) return fail(VEMB_E_INVALID, "set_state needs every array");
    if (!all_finite(it.host, it.count)) return fail(VEMB_E_NUMERIC, "set_state: non-finite entries");
  }
  const size_t vm = (size_t)2 * p->Ku * p->n_op * p->n_op;
  const bool with_v = st->Vpair && st->Vmom;
  if (with_v && (!all_finite(st->Vpair, P * n2) || !all_finite(st->Vmom, vm)))
    return fail(VEMB_E_NUMERIC, "set_state: non-finite eigenvectors");
  hipStream_t s = p->stream;
  for (const Item& it : items)
    VEMB_TRY(hip_rc(hipMemcpyAsync(it.dev, it.host, it.count * 8, hipMemcpyHostToDevice, s), "set_state copy"));
  if (with_v) {
    VEMB_TRY(hip_rc(hipMemcpyAsync(p->a.Vpair, st->Vpair, P * n2 * 8, hipMemcpyHostToDevice, s), "set_state V"));
    VEMB_TRY(hip_rc(hipMemcpyAsync(p->a.Vmom, st->Vmom, vm * 8, hipMemcpyHostToDevice, s), "set_state V"));
  }
  VEMB_TRY(hip_rc(hipStreamSynchronize(s), "set_state sync"));
  p->v_valid = with_v;
  p->k_valid = false;
  p->t = st->t;
  return VEMB_OK;
}

int vemb_penalties(const vemb_problem* p, double* mu, double* nu, double* eps, double* scale, double* last_feas,
                   double* last_gap) {
  if (!p) return fail(VEMB_E_INVALID, "NULL problem");
  if (mu) *mu = p->a.mu;
  if (nu) *nu = p->a.nu;
  if (eps) *eps = p->a.eps;
  if (scale) *scale = p->adapt_scale;
  if (last_feas) *last_feas = p->adapt_last;
  if (last_gap) *last_gap = p->adapt_last_gap;
  return VEMB_OK;
}

int vemb_set_penalty_scale(vemb_problem* p, double scale, double last_feas, double last_gap) {
  if (!p) return fail(VEMB_E_INVALID, "NULL problem");
  if (!(scale >= 1.0 && scale <= kAdaptMax)) return fail(VEMB_E_INVALID, "penalty scale outside [1, 8]");
  const bool have = last_feas >= 0.0 && last_gap >= 0.0;
  p->adapt_scale = scale;
  p->adapt_last = have ? last_feas : -1.0;
  p->adapt_last_gap = have ? last_gap : -1.0;
  set_parameters(p->a, scale * p->opt.mu, scale * p->opt.nu, scale * p->opt.eps);
  return VEMB_OK;
}

int vemb_divergence_check(const double* feas, int count, double lb, double energy) {
  if (!feas || count < 1) return fail(VEMB_E_INVALID, "vemb_divergence_check needs at least one value");
  const double last = feas[count - 1];
  if (!std::isfinite(lb) || !std::isfinite(energy) || !std::isfinite(last))
    return fail(VEMB_E_NUMERIC, "non-finite bound, energy or feasibility error");
  if (last > 1e3) return fail(VEMB_E_DIVERGED, "feasibility error " + std::to_string(last) + " above 1e3");
  constexpr int kRises = 5;
  if (count > kRises) {
    bool rising = true;
    for (int i = count - kRises; i < count; ++i) rising = rising && feas[i] > feas[i - 1];
    double lo = feas[0];
    for (int i = 1; i < count; ++i) lo = std::min(lo, feas[i]);
    if (rising && last >= 100.0 * lo)
      return fail(VEMB_E_DIVERGED, "feasibility error rose at each of the last 5 checks to " + std::to_string(last) +
                                       ", 100 times its smallest value");
  }
  return VEMB_OK;
}

int vemb_tuned_threads(int n, int is_complex, int precision, int batch, void* hip_stream) {
  if (n <= 0 || batch <= 0) return fail(VEMB_E_INVALID, "bad arguments to vemb_tuned_threads");
  return tuned_tpb(n, is_complex != 0, precision, batch, static_cast<hipStream_t>(hip_stream));
}

int vemb_problem_threads(const vemb_problem* p, int* pair_tpb, int* momentum_tpb) {
  if (!p) return fail(VEMB_E_INVALID, "NULL problem");
  if (pair_tpb) *pair_tpb = p->tpb_pair;
  if (momentum_tpb) *momentum_tpb = p->tpb_mom;
  return VEMB_OK;
}

int vemb_last_sweeps(vemb_problem* p, int* pair_max, int* momentum_max) {
  if (!p) return fail(VEMB_E_INVALID, "NULL problem");
  std::vector<int> sw(p->P + p->Ku);
  VEMB_TRY(hip_rc(hipMemcpyAsync(sw.data(), p->a.sweeps, sw.size() * sizeof(int), hipMemcpyDeviceToHost, p->stream),
                  "copy sweeps"));
  VEMB_TRY(hip_rc(hipStreamSynchronize(p->stream), "sweeps sync"));
  int a = 0, b = 0;
  for (int i = 0; i < p->P; ++i) a = std::max(a, sw[i]);
  for (int i = 0; i < p->Ku; ++i) b = std::max(b, sw[p->P + i]);
  if (pair_max) *pair_max = a;
  if (momentum_max) *momentum_max = b;
  if (std::max(a, b) > p->opt.max_sweeps)
    return fail(VEMB_E_NOCONV, "an eigensolve stopped at the sweep cap of " + std::to_string(p->opt.max_sweeps) +
                                   " unconverged (its next solve starts cold)");
  return VEMB_OK;
}

int vemb_set_profiling(vemb_problem* p, int enable) {
  if (!p) return fail(VEMB_E_INVALID, "NULL problem");
  VEMB_TRY(drain_marks(p));
  for (int k = 0; k < VEMB_K_COUNT; ++k) {
    p->prof_ms[k] = 0.0;
    p->prof_n[k] = 0;
  }
  p->profiling = enable != 0;
  p->prof_mask = enable ? 0xffffffffu : 0u;
  // events for the timings are created here, not between launches
  while (p->profiling && p->free_events.size() < 2048) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) break;
    p->free_events.push_back(e);
  }
  return VEMB_OK;
}

int vemb_set_profiling_mask(vemb_problem* p, uint32_t kernels) {
  VEMB_TRY(vemb_set_profiling(p, kernels != 0));
  p->prof_mask = kernels;
  return VEMB_OK;
}

int vemb_set_profiling_every(vemb_problem* p, int every) {
  if (!p || every < 1) return fail(VEMB_E_INVALID, "bad arguments to vemb_set_profiling_every");
  p->prof_every = every;
  return VEMB_OK;
}

int vemb_get_profile(vemb_problem* p, vemb_profile* out) {
  if (!p || !out) return fail(VEMB_E_INVALID, "NULL argument");
  VEMB_TRY(drain_marks(p));
  for (int k = 0; k < VEMB_K_COUNT; ++k) {
    out->ms[k] = p->prof_ms[k];
    out->launches[k] = p->prof_n[k];
  }
  return VEMB_OK;
}

void vemb_destroy(vemb_problem* p) {
  if (!p) return;
  if (p->stream) hipStreamSynchronize(p->stream);
  else hipDeviceSynchronize();
  for (auto& mk : p->marks) {
    hipEventDestroy(mk.start);
    hipEventDestroy(mk.stop);
  }
  for (hipEvent_t e : p->free_events) hipEventDestroy(e);
  p->mem.release();
  if (p->diag_ev) hipEventDestroy(p->diag_ev);
  if (p->diag_host) hipHostFree(p->diag_host);
  if (p->fork_ev) hipEventDestroy(p->fork_ev);
  if (p->join_ev) hipEventDestroy(p->join_ev);
  if (p->side) hipStreamDestroy(p->side);
  delete p;
  object_destroyed();
}

int vemb_psd_project_batched(const double* in, double* out, int n, int batch, int is_complex, int precision,
                             void* hip_stream) {
  return vemb_psd_project_batched_ex(in, out, n, batch, is_complex, precision, 0, nullptr, 0, hip_stream);
}

namespace {
// Large matrices (streamed solver) need per-matrix scratch: allocated for the call,
// freed after the stream drains (these calls synchronise).
struct Scratch {
  DeviceMemory mem;
  void* w = nullptr;
  void* t = nullptr;
  void* v = nullptr;
  ~Scratch() { mem.release(); }
};
}  // namespace

int vemb_psd_project_batched_ex(const double* in, double* out, int n, int batch, int is_complex, int precision,
                                int max_sweeps, int* sweeps, int tpb, void* hip_stream) {
  if (!in || !out || n <= 0 || batch < 0) return fail(VEMB_E_INVALID, "bad arguments to vemb_psd_project_batched_ex");
  if (precision < VEMB_FP64 || precision > VEMB_FP32) return fail(VEMB_E_INVALID, "unknown precision");
  if (n > 256) return fail(VEMB_E_UNSUPPORTED, "matrices above 256 x 256 are not supported");
  const int ms = max_sweeps > 0 ? max_sweeps : 40;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const bool lds = (is_complex && n <= 64) || (!is_complex && n <= 128);
  const bool need_v = precision == VEMB_MIXED && !(n > 64 && n <= 128);  // MIXED keeps eigenvectors between passes
  const size_t bytes = (size_t)batch * n * n * (is_complex ? 16 : 8);
  Scratch sc;
  if (need_v && !(sc.v = sc.mem.get(bytes))) return fail(VEMB_E_NOMEM, "eigenvector scratch");
  if (lds) {
    const int t = tpb > 0 ? tpb : tuned_tpb(n, is_complex != 0, precision, batch, st);
    VEMB_TRY(hip_rc(launch_psd_batched(in, out, n, batch, is_complex != 0, precision, ms, sweeps, (double*)sc.v, t,
                                       st),
                    "batched projection"));
    return sc.v ? hip_rc(hipStreamSynchronize(st), "batched projection sync") : VEMB_OK;
  }
  if (n % 32) return fail(VEMB_E_UNSUPPORTED, "streamed solver needs n divisible by 32");
  if (!(sc.w = sc.mem.get(bytes)) || !(sc.t = sc.mem.get(bytes)))
    return fail(VEMB_E_NOMEM, "scratch for the streamed solver");
  VEMB_TRY(hip_rc(launch_psd_batched_big(in, out, n, batch, is_complex != 0, precision, ms, sweeps, (double*)sc.v,
                                         sc.w, sc.t, st),
                  "batched projection"));
  return hip_rc(hipStreamSynchronize(st), "batched projection sync");
}

int vemb_psd_project_sign(const double* in, double* out, int n, void* hip_stream) {
  if (!in || !out) return fail(VEMB_E_INVALID, "NULL argument");
  if (n <= 0 || n % 16 || n > 4096) return fail(VEMB_E_INVALID, "n must be a positive multiple of 16, at most 4096");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  DeviceMemory mem;
  const size_t words = 4 * (size_t)n * n + 64;
  double* work = static_cast<double*>(mem.get(words * sizeof(double)));
  if (!work) return fail(VEMB_E_NOMEM, "sign-projection scratch");
  int rc = hip_rc(launch_psd_project_ns(in, out, n, work, ns_schedule(kNsResolved), st), "sign projection");
  if (rc == VEMB_OK) rc = hip_rc(hipStreamSynchronize(st), "sign projection sync");
  hipStreamSynchronize(st);  // the scratch goes back only after the stream has drained
  mem.release();
  return rc;
}

int vemb_psd_project_sign_noalloc(const double* in, double* out, int n, void* hip_stream) {
  if (!in || !out) return fail(VEMB_E_INVALID, "NULL argument");
  if (n <= 0 || n % 16) return fail(VEMB_E_INVALID, "n must be a positive multiple of 16");
  if (n > kStaticSignMaxN)
    return fail(VEMB_E_INVALID, "n = " + std::to_string(n) + " exceeds the static scratch limit of " +
                                    std::to_string(kStaticSignMaxN));
  double* work = nullptr;
  VEMB_TRY(hip_rc(static_sign_scratch(&work), "static scratch address"));
  return hip_rc(launch_psd_project_ns(in, out, n, work, ns_schedule_resolved(), static_cast<hipStream_t>(hip_stream)),
                "sign projection");
}

int vemb_tile_map(int kind, int n, int count, int* grid, int* map) {
  if (!grid) return fail(VEMB_E_INVALID, "NULL grid");
  int g = 0;
  if (kind == 0) {
    if (n <= 0 || n % 16 || n > 4096) return fail(VEMB_E_INVALID, "kind 0: n a positive multiple of 16, at most 4096");
    g = upper_tile_count(n / 16);
  } else if (kind == 1) {
    if (n <= 0 || n % 64 || n > kSignMax || count <= 0)
      return fail(VEMB_E_INVALID, "kind 1: n a positive multiple of 64 up to 256, count > 0");
    g = upper_tile_count(n / 64) * count;
  } else {
    return fail(VEMB_E_INVALID, "kind must be 0 or 1");
  }
  *grid = g;
  if (!map) return VEMB_OK;
  for (int w = 0; w < g; ++w) {
    int b = 0, ti = -1, tj = -1;
    const int tu = upper_tile_count(n / 64);  // kind 1: grid (tu, count), linear index bx + tu * by
    const bool live = kind == 0 ? upper_tile(w, n / 16, &ti, &tj)
                                : batched_tile_of(w % tu, w / tu, count, n / 64, &b, &ti, &tj);
    map[4 * w] = live ? 1 : 0;
    map[4 * w + 1] = live ? b : -1;
    map[4 * w + 2] = live ? ti : -1;
    map[4 * w + 3] = live ? tj : -1;
  }
  return VEMB_OK;
}

int vemb_eigvalsh_batched(const double* in, double* w, int n, int batch, int is_complex, void* hip_stream) {
  if (!in || !w || n <= 0 || batch < 0) return fail(VEMB_E_INVALID, "bad arguments to vemb_eigvalsh_batched");
  if (n > 256) return fail(VEMB_E_UNSUPPORTED, "matrices above 256 x 256 are not supported");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if ((is_complex && n <= 64) || (!is_complex && n <= 128))
    return hip_rc(launch_eigvalsh_batched(in, w, n, batch, is_complex != 0, 40, nullptr, st), "batched eigenvalues");
  if (n % 32) return fail(VEMB_E_UNSUPPORTED, "streamed solver needs n divisible by 32");
  Scratch sc;
  const size_t bytes = (size_t)batch * n * n * (is_complex ? 16 : 8);
  if (!(sc.w = sc.mem.get(bytes)) || !(sc.t = sc.mem.get(bytes)))
    return fail(VEMB_E_NOMEM, "scratch for the streamed solver");
  VEMB_TRY(hip_rc(launch_eigvals_big(in, w, nullptr, n, batch, is_complex != 0, 40, nullptr, sc.w, sc.t, st),
                  "batched eigenvalues"));
  return hip_rc(hipStreamSynchronize(st), "batched eigenvalues sync");
}

}  // extern "C"

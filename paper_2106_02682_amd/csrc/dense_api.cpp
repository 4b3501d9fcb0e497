// C ABI of the dense Algorithm 5 solver (declared in include/vemb.h): one marginal per
// cluster and per unordered cluster pair, one dense dual X (Section 3.2), so that the
// cluster Hamiltonians may differ from cluster to cluster (one-site fields, disorder).
// The bonds stay those of a translation-invariant term list on the torus.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "alloc.h"
#include "dense.h"
#include "polar.h"
#include "problem.h"

using namespace vemb;

struct vemb_dense {
  Geometry g;
  int Q = 0, k = 0, ld = 0;
  vemb_options opt{};
  hipStream_t stream = nullptr, side = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  int64_t t = 0;
  bool v_valid = false;
  int tpb_pair = 256, tpb_x = 256;
  OpTables ops_host{};
  std::vector<int2> pairs_host;
  DenseArgs a{};
  DeviceMemory mem;  // every device allocation of the dense problem
  double* lmin = nullptr;   // Q + M smallest eigenvalues of the bound matrices
  double* feas = nullptr;   // Q: ||rho_ij - rho~_ij||^2 from the pair projection
  int* sweeps = nullptr;    // Q pair projections, then the X projection
  double* Vpair = nullptr;  // Q x n x n eigenvectors kept for the warm start
  double* Vx = nullptr;     // ld x ld (K <= 64: kept eigenvectors of the X projection)
  double* ns_work = nullptr;  // K > 64: scratch of the matrix-sign projection (4 ld^2 + 64)
  std::vector<double> ns_sched;
  void *wscr_pair = nullptr, *tscr_pair = nullptr;
};

namespace {

template <typename T>
int dalloc(vemb_dense* d, T** ptr, size_t count) {
  const size_t bytes = count == 0 ? 16 : count * sizeof(T);
  void* raw = d->mem.get(bytes);
  if (!raw) return fail(VEMB_E_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  *ptr = static_cast<T*>(raw);
  return VEMB_OK;
}

bool valid_tpb(int t) { return t == kTpbRegister8 || t == kTpbRegister4 || t == 256 || t == 512 || t == 1024; }

// Section 4's starting point: multipliers 0, marginals identity / trace, X = I.
int upload_initial(vemb_dense* d) {
  const DenseArgs& a = d->a;
  const int m = a.m, n = a.n, M = a.M, Q = a.Q;
  hipStream_t s = d->stream;
  std::vector<double> X((size_t)a.ld * a.ld, 0.0);
  for (int i = 0; i < a.K; ++i) X[(size_t)i * a.ld + i] = 1.0;
  std::vector<double> r0((size_t)M * m * m, 0.0);
  for (int c = 0; c < M; ++c)
    for (int i = 0; i < m; ++i) r0[(size_t)c * m * m + (size_t)i * m + i] = 1.0 / m;
  std::vector<double> rt((size_t)Q * n * n, 0.0);
  for (int e = 0; e < Q; ++e)
    for (int i = 0; i < n; ++i) rt[(size_t)e * n * n + (size_t)i * n + i] = 1.0 / n;
  VEMB_TRY(hip_rc(hipMemcpyAsync(a.X, X.data(), X.size() * 8, hipMemcpyHostToDevice, s), "upload X"));
  VEMB_TRY(hip_rc(hipMemsetAsync(a.Xp, 0, X.size() * 8, s), "zero X'"));
  VEMB_TRY(hip_rc(hipMemcpyAsync(a.rho0, r0.data(), r0.size() * 8, hipMemcpyHostToDevice, s), "upload rho0"));
  VEMB_TRY(hip_rc(hipMemcpyAsync(a.rho_t, rt.data(), rt.size() * 8, hipMemcpyHostToDevice, s), "upload rho_t"));
  VEMB_TRY(hip_rc(hipMemcpyAsync(a.rho, rt.data(), rt.size() * 8, hipMemcpyHostToDevice, s), "upload rho"));
  VEMB_TRY(hip_rc(hipMemsetAsync(a.Lam, 0, (size_t)Q * n * n * 8, s), "zero Lam"));
  VEMB_TRY(hip_rc(hipMemsetAsync(a.Lam1, 0, (size_t)Q * m * m * 8, s), "zero Lam1"));
  VEMB_TRY(hip_rc(hipMemsetAsync(a.Lam2, 0, (size_t)Q * m * m * 8, s), "zero Lam2"));
  VEMB_TRY(hip_rc(hipMemsetAsync(a.e_pair, 0, (size_t)Q * 8, s), "zero e_pair"));
  VEMB_TRY(hip_rc(hipMemsetAsync(a.e_clu, 0, (size_t)M * 8, s), "zero e_clu"));
  VEMB_TRY(hip_rc(hipMemsetAsync(a.cons, 0, (size_t)Q * 8, s), "zero cons"));
  VEMB_TRY(hip_rc(hipMemsetAsync(d->feas, 0, (size_t)Q * 8, s), "zero feas"));
  VEMB_TRY(hip_rc(hipMemsetAsync(d->sweeps, 0, (size_t)(Q + 1) * sizeof(int), s), "zero sweeps"));
  VEMB_TRY(hip_rc(hipStreamSynchronize(s), "initial upload"));
  d->t = 0;
  d->v_valid = false;
  return VEMB_OK;
}

int copy_back(vemb_dense* d, std::vector<double>& h, const double* src, size_t count) {
  h.resize(count);
  VEMB_TRY(hip_rc(hipMemcpyAsync(h.data(), src, count * 8, hipMemcpyDeviceToHost, d->stream), "copy back"));
  return VEMB_OK;
}

double sum_of(const std::vector<double>& v) {
  double s = 0.0;
  for (double x : v) s += x;
  return s;
}

}  // namespace

extern "C" {

int vemb_dense_create(const vemb_hamiltonian* H, const vemb_lattice* lat, const vemb_clusters* cl,
                      const vemb_site_field* fields, int nfields, const vemb_options* opts, void* hip_stream,
                      vemb_dense** out) {
  if (!H || !lat || !cl || !out || (H->nterms > 0 && !H->terms) || nfields < 0 || (nfields > 0 && !fields))
    return fail(VEMB_E_INVALID, "NULL argument");
  *out = nullptr;
  vemb_options o;
  Geometry g{};
  std::string err;
  int rc = normalize_options(opts, o, err);
  if (rc == VEMB_OK) rc = parse_geometry(*lat, *cl, g, err);
  if (rc != VEMB_OK) return fail(rc, err);
  const int m = g.m, n = g.n, M = g.M;
  const int k = o.opset == VEMB_OPSET_COMPLETE ? n : 3 * g.L;
  const int K = M * k;
  // the dense projection is one K x K problem: LDS Jacobi up to 64, matrix-sign iteration on
  // matrix cores above (storage padded with zeros to a multiple of 32)
  if (K > 1024) return fail(VEMB_E_UNSUPPORTED, "dense X above 1024 x 1024 (M n_op = " + std::to_string(K) + ")");
  if (n > 256) return fail(VEMB_E_UNSUPPORTED, "pair matrices above 256 x 256 are not supported");
  if (o.adapt_every > 0) return fail(VEMB_E_UNSUPPORTED, "adaptive parameters run on translation-invariant problems");
  const int ld = K <= 64 ? K : (K + 31) / 32 * 32;
  HostModel host;
  rc = build_model(*H, g, host, err, o.fermionic != 0);
  if (rc != VEMB_OK) return fail(rc, err);
  std::vector<double> Hc((size_t)M * m * m);
  for (int c = 0; c < M; ++c)
    for (size_t e = 0; e < (size_t)m * m; ++e) Hc[(size_t)c * m * m + e] = host.H0[e];
  for (int f = 0; f < nfields; ++f) {
    if (o.fermionic && fields[f].pauli != VEMB_Z)
      return fail(VEMB_E_UNSUPPORTED, "field " + std::to_string(f) + ": fermionic fields are Z (1 - 2n)");
    rc = add_site_field(g, fields[f].x, fields[f].y, fields[f].pauli, fields[f].coeff, Hc, err);
    if (rc != VEMB_OK) return fail(rc, "field " + std::to_string(f) + ": " + err);
  }

  auto* d = new vemb_dense();
  object_created();
  d->g = g;
  d->k = k;
  d->ld = ld;
  d->opt = o;
  d->stream = static_cast<hipStream_t>(hip_stream);
  for (int i = 0; i < M; ++i)
    for (int j = i + 1; j < M; ++j) d->pairs_host.push_back(int2{i, j});
  const int Q = (int)d->pairs_host.size();
  d->Q = Q;
  // H_ij is the interaction of clusters i and j: H_0d of the offset d = j - i on the torus
  std::vector<int> hp_index(Q);
  for (int e = 0; e < Q; ++e) {
    const int i = d->pairs_host[e].x, j = d->pairs_host[e].y;
    const int ix = i / g.My, iy = i % g.My, jx = j / g.My, jy = j % g.My;
    const int off = ((jx - ix + g.Mx) % g.Mx) * g.My + ((jy - iy + g.My) % g.My);
    hp_index[e] = host.hd_index[off - 1];
  }
  if (o.opset == VEMB_OPSET_PAULI1) build_pauli1_tables(g.L, d->ops_host);
  DenseArgs& a = d->a;
  a.M = M;
  a.Q = Q;
  a.m = m;
  a.n = n;
  a.k = k;
  a.K = K;
  a.ld = ld;
  a.opset = o.opset;
  a.fermionic = o.fermionic;
  a.mu = o.mu;
  a.nu = o.nu;
  a.eps = o.eps;
  a.sign = o.sign < 0 ? -1.0 : 1.0;
  a.a = 1.0 / o.mu;
  a.b = 1.0 / (o.mu + o.nu * m) - 1.0 / o.mu;
  a.c = 1.0 / (o.mu + 2 * o.nu * m) - 2.0 / (o.mu + o.nu * m) + 1.0 / o.mu;
  auto cleanup = [&](int code) {
    vemb_dense_destroy(d);
    return code;
  };
  if (hipStreamCreateWithFlags(&d->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&d->fork_ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&d->join_ev, hipEventDisableTiming) != hipSuccess)
    return cleanup(fail(VEMB_E_HIP, "side stream / events"));
  const size_t nh = host.Hd.size() / ((size_t)n * n);
  int2* pairs_dev = nullptr;
  double *Hc_dev = nullptr, *Hp_dev = nullptr;
  int* hpi_dev = nullptr;
  OpTables* ops_dev = nullptr;
  const size_t nn = (size_t)n * n, mm = (size_t)m * m, xx = (size_t)ld * ld;
  if ((rc = dalloc(d, &pairs_dev, Q)) || (rc = dalloc(d, &Hc_dev, M * mm)) || (rc = dalloc(d, &Hp_dev, nh * nn)) ||
      (rc = dalloc(d, &hpi_dev, Q)) || (rc = dalloc(d, &ops_dev, 1)) || (rc = dalloc(d, &a.X, xx)) ||
      (rc = dalloc(d, &a.Xp, xx)) || (rc = dalloc(d, &a.rho0, M * mm)) || (rc = dalloc(d, &a.rho, Q * nn)) ||
      (rc = dalloc(d, &a.rho_t, Q * nn)) || (rc = dalloc(d, &a.Lam, Q * nn)) || (rc = dalloc(d, &a.Lam1, Q * mm)) ||
      (rc = dalloc(d, &a.Lam2, Q * mm)) || (rc = dalloc(d, &a.tr2, Q * mm)) || (rc = dalloc(d, &a.tr1, Q * mm)) ||
      (rc = dalloc(d, &a.e_pair, Q)) || (rc = dalloc(d, &a.e_clu, M)) || (rc = dalloc(d, &a.cons, Q)) ||
      (rc = dalloc(d, &a.Kbuf, Q * nn + M * mm)) || (rc = dalloc(d, &d->lmin, (size_t)Q + M)) ||
      (rc = dalloc(d, &d->feas, Q)) || (rc = dalloc(d, &d->sweeps, (size_t)Q + 1)) ||
      (rc = dalloc(d, &d->Vpair, Q * nn)) || (ld <= 64 && (rc = dalloc(d, &d->Vx, xx))) ||
      (n > 64 && ((rc = dalloc(d, (double**)&d->wscr_pair, Q * nn)) || (rc = dalloc(d, (double**)&d->tscr_pair, Q * nn)))) ||
      (ld > 64 && (rc = dalloc(d, &d->ns_work, 4 * xx + 64))))
    return cleanup(rc);
  hipStream_t s = d->stream;
  if ((rc = hip_rc(hipMemcpyAsync(pairs_dev, d->pairs_host.data(), Q * sizeof(int2), hipMemcpyHostToDevice, s), "upload pairs")) ||
      (rc = hip_rc(hipMemcpyAsync(Hc_dev, Hc.data(), Hc.size() * 8, hipMemcpyHostToDevice, s), "upload H_i")) ||
      (nh && (rc = hip_rc(hipMemcpyAsync(Hp_dev, host.Hd.data(), host.Hd.size() * 8, hipMemcpyHostToDevice, s), "upload H_ij"))) ||
      (rc = hip_rc(hipMemcpyAsync(hpi_dev, hp_index.data(), Q * sizeof(int), hipMemcpyHostToDevice, s), "upload index")) ||
      (rc = hip_rc(hipMemcpyAsync(ops_dev, &d->ops_host, sizeof(OpTables), hipMemcpyHostToDevice, s), "upload ops")))
    return cleanup(rc);
  a.pairs = pairs_dev;
  a.Hc = Hc_dev;
  a.Hp = Hp_dev;
  a.hp_index = hpi_dev;
  a.ops = ops_dev;
  if ((rc = upload_initial(d))) return cleanup(rc);
  if (ld > 64) d->ns_sched = ns_schedule(kNsResolved);
  if (valid_tpb(o.tpb)) {
    d->tpb_pair = d->tpb_x = o.tpb;
  } else {
    if (n <= 64) d->tpb_pair = tuned_tpb(n, false, o.precision, Q, s);
    if (ld <= 64) d->tpb_x = tuned_tpb(ld, false, o.precision, 1, s);
  }
  *out = d;
  return VEMB_OK;
}

int vemb_dense_get_info(const vemb_dense* d, vemb_dense_info* info) {
  if (!d || !info) return fail(VEMB_E_INVALID, "NULL argument");
  info->M = d->g.M;
  info->Q = d->Q;
  info->L = d->g.L;
  info->m = d->g.m;
  info->n = d->g.n;
  info->n_op = d->k;
  info->K = d->a.K;
  info->t = d->t;
  return VEMB_OK;
}

int vemb_dense_step(vemb_dense* d, int iters) {
  if (!d || iters < 0) return fail(VEMB_E_INVALID, "NULL problem or negative iteration count");
  const DenseArgs& a = d->a;
  hipStream_t s = d->stream, s2 = d->side;
  const int ms = d->opt.max_sweeps, prec = d->opt.precision;
  for (int it = 0; it < iters; ++it) {
    const int refresh = d->opt.warm_refresh;
    const int cold = (!d->v_valid || refresh < 0 || d->t % refresh == 0) ? 1 : 0;
    VEMB_TRY(hip_rc(launch_dense_pair_update(a, s), "dense pair update"));
    // the pair projection (rho~, Lambda) feeds only the next iteration: side stream
    VEMB_TRY(hip_rc(hipEventRecord(d->fork_ev, s), "fork"));
    VEMB_TRY(hip_rc(hipStreamWaitEvent(s2, d->fork_ev, 0), "fork"));
    VEMB_TRY(hip_rc(a.n > 64 ? launch_pair_projection_big(a.rho, a.Lam, a.rho_t, d->feas, a.n, a.Q, a.mu, prec, ms,
                                                          d->sweeps, d->Vpair, cold, d->wscr_pair, d->tscr_pair, s2)
                             : launch_pair_projection(a.rho, a.Lam, a.rho_t, d->feas, a.n, a.Q, a.mu, prec, ms,
                                                      d->sweeps, d->Vpair, cold, d->tpb_pair, s2),
                    "dense pair projection"));
    VEMB_TRY(hip_rc(hipEventRecord(d->join_ev, s2), "join"));
    VEMB_TRY(hip_rc(launch_dense_cluster(a, s), "dense cluster update"));
    VEMB_TRY(hip_rc(launch_dense_xstep(a, s), "dense X step"));
    VEMB_TRY(hip_rc(a.ld > 64 ? launch_psd_project_ns(a.Xp, a.X, a.ld, d->ns_work, d->ns_sched, s)
                              : launch_psd_batched(a.Xp, a.X, a.ld, 1, false, prec, ms, d->sweeps + a.Q, d->Vx,
                                                   d->tpb_x, s, cold),
                    "dense X projection"));
    VEMB_TRY(hip_rc(hipStreamWaitEvent(s, d->join_ev, 0), "join"));
    d->v_valid = true;
    ++d->t;
  }
  return VEMB_OK;
}

int vemb_dense_dual_bound(vemb_dense* d, double* lb_per_site) {
  if (!d || !lb_per_site) return fail(VEMB_E_INVALID, "NULL argument");
  const DenseArgs& a = d->a;
  hipStream_t s = d->stream;
  const int ms = d->opt.max_sweeps;
  VEMB_TRY(hip_rc(launch_dense_bound_build(a, s), "dense bound build"));
  VEMB_TRY(hip_rc(a.n > 128 ? launch_eigvals_big(a.Kbuf, nullptr, d->lmin, a.n, a.Q, false, ms, nullptr, d->wscr_pair,
                                                  d->tscr_pair, s)
                            : launch_lambda_min(a.Kbuf, d->lmin, a.n, a.Q, ms, nullptr, s),
                  "pair lambda_min"));
  VEMB_TRY(hip_rc(launch_lambda_min(a.Kbuf + (size_t)a.Q * a.n * a.n, d->lmin + a.Q, a.m, a.M, ms, nullptr, s),
                  "cluster lambda_min"));
  std::vector<double> lm;
  VEMB_TRY(copy_back(d, lm, d->lmin, (size_t)a.Q + a.M));
  VEMB_TRY(hip_rc(hipStreamSynchronize(s), "bound sync"));
  const double v = sum_of(lm) / ((double)a.M * d->g.L);
  if (!std::isfinite(v)) return fail(VEMB_E_NUMERIC, "non-finite dual bound");
  *lb_per_site = v;
  return VEMB_OK;
}

int vemb_dense_primal_energy(vemb_dense* d, double* e_per_site, double* feas_err) {
  if (!d || (!e_per_site && !feas_err)) return fail(VEMB_E_INVALID, "NULL argument");
  const DenseArgs& a = d->a;
  std::vector<double> ep, ec, fe, co;
  VEMB_TRY(copy_back(d, ep, a.e_pair, a.Q));
  VEMB_TRY(copy_back(d, ec, a.e_clu, a.M));
  VEMB_TRY(copy_back(d, fe, d->feas, a.Q));
  VEMB_TRY(copy_back(d, co, a.cons, a.Q));
  VEMB_TRY(hip_rc(hipStreamSynchronize(d->stream), "energy sync"));
  if (e_per_site) *e_per_site = (sum_of(ep) + sum_of(ec)) / ((double)a.M * d->g.L);
  if (feas_err) *feas_err = std::sqrt((sum_of(fe) + sum_of(co)) / a.M);
  return VEMB_OK;
}

int vemb_dense_get_state(vemb_dense* d, vemb_dense_state* st) {
  if (!d || !st) return fail(VEMB_E_INVALID, "NULL argument");
  const DenseArgs& a = d->a;
  hipStream_t s = d->stream;
  const size_t nn = (size_t)a.n * a.n, mm = (size_t)a.m * a.m;
  if (st->X)
    VEMB_TRY(hip_rc(hipMemcpy2DAsync(st->X, (size_t)a.K * 8, a.X, (size_t)a.ld * 8, (size_t)a.K * 8, a.K,
                                     hipMemcpyDeviceToHost, s),
                    "copy X"));
  struct Item { double* dst; const double* src; size_t count; };
  const Item items[] = {{st->rho0, a.rho0, a.M * mm}, {st->rho, a.rho, a.Q * nn},  {st->rho_t, a.rho_t, a.Q * nn},
                        {st->Lam, a.Lam, a.Q * nn},   {st->Lam1, a.Lam1, a.Q * mm}, {st->Lam2, a.Lam2, a.Q * mm}};
  for (const Item& it : items)
    if (it.dst) VEMB_TRY(hip_rc(hipMemcpyAsync(it.dst, it.src, it.count * 8, hipMemcpyDeviceToHost, s), "copy state"));
  VEMB_TRY(hip_rc(hipStreamSynchronize(s), "state sync"));
  st->t = d->t;
  return VEMB_OK;
}

int vemb_dense_set_state(vemb_dense* d, const vemb_dense_state* st) {
  if (!d || !st) return fail(VEMB_E_INVALID, "NULL argument");
  const DenseArgs& a = d->a;
  hipStream_t s = d->stream;
  const size_t nn = (size_t)a.n * a.n, mm = (size_t)a.m * a.m;
  struct Item { const double* src; double* dst; size_t count; };
  const Item items[] = {{st->X, nullptr, (size_t)a.K * a.K},  {st->rho0, a.rho0, a.M * mm},
                        {st->rho, a.rho, a.Q * nn},            {st->rho_t, a.rho_t, a.Q * nn},
                        {st->Lam, a.Lam, a.Q * nn},            {st->Lam1, a.Lam1, a.Q * mm},
                        {st->Lam2, a.Lam2, a.Q * mm}};
  for (const Item& it : items)
    if (it.src)
      for (size_t i = 0; i < it.count; ++i)
        if (!std::isfinite(it.src[i])) return fail(VEMB_E_NUMERIC, "non-finite value in the state");
  if (st->X)
    VEMB_TRY(hip_rc(hipMemcpy2DAsync(a.X, (size_t)a.ld * 8, st->X, (size_t)a.K * 8, (size_t)a.K * 8, a.K,
                                     hipMemcpyHostToDevice, s),
                    "upload X"));
  for (const Item& it : items)
    if (it.src && it.dst)
      VEMB_TRY(hip_rc(hipMemcpyAsync(it.dst, it.src, it.count * 8, hipMemcpyHostToDevice, s), "upload state"));
  VEMB_TRY(hip_rc(hipStreamSynchronize(s), "state sync"));
  d->t = st->t;
  d->v_valid = false;
  return VEMB_OK;
}

int vemb_dense_last_sweeps(vemb_dense* d, int* pair_max, int* x_sweeps) {
  if (!d) return fail(VEMB_E_INVALID, "NULL argument");
  std::vector<int> sw((size_t)d->Q + 1);
  VEMB_TRY(hip_rc(hipMemcpyAsync(sw.data(), d->sweeps, sw.size() * sizeof(int), hipMemcpyDeviceToHost, d->stream),
                  "copy sweeps"));
  VEMB_TRY(hip_rc(hipStreamSynchronize(d->stream), "sweeps sync"));
  int mx = 0;
  for (int e = 0; e < d->Q; ++e) mx = sw[e] > mx ? sw[e] : mx;
  if (pair_max) *pair_max = mx;
  if (x_sweeps) *x_sweeps = d->ld > 64 ? (int)d->ns_sched.size() : sw[d->Q];
  return VEMB_OK;
}

void vemb_dense_destroy(vemb_dense* d) {
  if (!d) return;
  if (d->stream) hipStreamSynchronize(d->stream);
  if (d->side) hipStreamSynchronize(d->side);
  d->mem.release();
  if (d->fork_ev) hipEventDestroy(d->fork_ev);
  if (d->join_ev) hipEventDestroy(d->join_ev);
  if (d->side) hipStreamDestroy(d->side);
  delete d;
  object_destroyed();
}

}  // extern "C"

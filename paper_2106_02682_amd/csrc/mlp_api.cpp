// C ABI of the learned warm start's network (vemb_mlp_*): parameter storage,
// forward / backward / Adam on the device, normalisation of the targets.
#include <cmath>
#include <vector>

#include "mlp.h"
#include "problem.h"

using namespace vemb;

struct vemb_mlp {
  std::vector<int> dims;  // dims[0] inputs ... dims.back() outputs
  int layers = 0;
  long nparams = 0;
  std::vector<long> offW, offB;
  int max_batch = 0;
  hipStream_t stream = nullptr;
  float *theta = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
  uint16_t* wbf = nullptr;
  float *mean = nullptr, *stdv = nullptr;
  std::vector<float*> Z, A;  // per layer, max_batch x dims[l+1]
  float *dZa = nullptr, *dZb = nullptr;  // ping-pong gradient buffers, max_batch x max width
  float *xb = nullptr, *tb = nullptr;    // gathered minibatch
  double* partial = nullptr;
  double* loss = nullptr;
  float* ws = nullptr;  // split-K workspace
  long ws_floats = 0;
  int64_t t = 0;
  vemb::DeviceMemory mem;  // every device allocation of the network
};

namespace {

constexpr int kMaxPartials = 1024;
constexpr int kSplitSlices = 64;

template <typename T>
int malloc_into(vemb_mlp* n, T** p, size_t count) {
  void* raw = n->mem.get(std::max<size_t>(count, 1) * sizeof(T));
  if (!raw) return fail(VEMB_E_NOMEM, "network allocation");
  *p = static_cast<T*>(raw);
  return VEMB_OK;
}

int forward_pass(vemb_mlp* n, const float* x, int B) {
  const float* a = x;
  for (int l = 0; l < n->layers; ++l) {
    const int in = n->dims[l], out = n->dims[l + 1];
    const bool hidden = l < n->layers - 1;
    GemmArgs g{};
    g.M = B;
    g.N = out;
    g.K = in;
    g.A = a;
    g.sai = in;
    g.sak = 1;
    g.B = n->wbf + n->offW[l];  // B(k, j) = W(j, k)
    g.sbk = 1;
    g.sbj = in;
    g.C = n->Z[l];
    g.ldc = out;
    g.bias = n->theta + n->offB[l];
    g.epi = hidden ? kEpiSilu : kEpiPlain;
    g.C2 = hidden ? n->A[l] : nullptr;
    g.ws = n->ws;
    g.ws_floats = n->ws_floats;
    VEMB_TRY(hip_rc(launch_gemm(g, true, n->stream), "network forward GEMM"));
    a = hidden ? n->A[l] : n->Z[l];
  }
  return VEMB_OK;
}

// Gradients of the mean squared error on normalised targets into n->grad; loss on the device.
int backward_pass(vemb_mlp* n, const float* x, const float* t, int B) {
  VEMB_TRY(forward_pass(n, x, B));
  const int L = n->layers, O = n->dims[L];
  float* dZ = n->dZa;
  float* dZn = n->dZb;
  VEMB_TRY(hip_rc(launch_loss_grad(n->Z[L - 1], t, n->mean, n->stdv, B, O, dZ, n->partial, kMaxPartials, n->loss,
                                   n->stream),
                  "network loss"));
  for (int l = L - 1; l >= 0; --l) {
    const int in = n->dims[l], out = n->dims[l + 1];
    const float* aprev = l > 0 ? n->A[l - 1] : x;
    GemmArgs gw{};  // dW = dZ^T A_{l-1}: (out x B)(B x in)
    gw.M = out;
    gw.N = in;
    gw.K = B;
    gw.A = dZ;
    gw.sai = 1;
    gw.sak = out;
    gw.B = aprev;
    gw.sbk = in;
    gw.sbj = 1;
    gw.C = n->grad + n->offW[l];
    gw.ldc = in;
    gw.epi = kEpiPlain;
    gw.ws = n->ws;
    gw.ws_floats = n->ws_floats;
    VEMB_TRY(hip_rc(launch_gemm(gw, false, n->stream), "network weight gradient"));
    VEMB_TRY(hip_rc(launch_colsum(dZ, B, out, n->grad + n->offB[l], n->stream), "network bias gradient"));
    if (l > 0) {
      GemmArgs gd{};  // dZ_{l-1} = (dZ W) * silu'(Z_{l-1}): (B x out)(out x in)
      gd.M = B;
      gd.N = in;
      gd.K = out;
      gd.A = dZ;
      gd.sai = out;
      gd.sak = 1;
      gd.B = n->wbf + n->offW[l];
      gd.sbk = in;
      gd.sbj = 1;
      gd.C = dZn;
      gd.ldc = in;
      gd.epi = kEpiSiluGrad;
      gd.Z = n->Z[l - 1];
      gd.ldz = in;
      gd.ws = n->ws;
      gd.ws_floats = n->ws_floats;
      VEMB_TRY(hip_rc(launch_gemm(gd, true, n->stream), "network backward GEMM"));
      std::swap(dZ, dZn);
    }
  }
  return VEMB_OK;
}

int check_batch(const vemb_mlp* n, int B) {
  if (B <= 0 || B > n->max_batch) return fail(VEMB_E_INVALID, "batch size outside 1..max_batch");
  return VEMB_OK;
}

int read_loss(vemb_mlp* n, double* loss_host) {
  if (!loss_host) return VEMB_OK;
  VEMB_TRY(hip_rc(hipMemcpyAsync(loss_host, n->loss, sizeof(double), hipMemcpyDeviceToHost, n->stream), "loss copy"));
  return hip_rc(hipStreamSynchronize(n->stream), "loss sync");
}

}  // namespace

extern "C" {

int vemb_mlp_create(const int32_t* dims, int n_dims, const float* params, int max_batch, void* hip_stream,
                    vemb_mlp** out) {
  if (!dims || n_dims < 2 || !out || max_batch <= 0) return fail(VEMB_E_INVALID, "bad arguments to vemb_mlp_create");
  *out = nullptr;
  for (int i = 0; i < n_dims; ++i)
    if (dims[i] <= 0) return fail(VEMB_E_INVALID, "layer widths must be positive");
  auto* n = new vemb_mlp();
  object_created();
  n->dims.assign(dims, dims + n_dims);
  n->layers = n_dims - 1;
  n->max_batch = max_batch;
  n->stream = static_cast<hipStream_t>(hip_stream);
  long o = 0;
  int wmax = 0;
  for (int l = 0; l < n->layers; ++l) {
    n->offW.push_back(o);
    o += (long)dims[l + 1] * dims[l];
    n->offB.push_back(o);
    o += dims[l + 1];
    wmax = std::max(wmax, std::max(dims[l], dims[l + 1]));
  }
  n->nparams = o;
  auto cleanup = [&](int rc) {
    vemb_mlp_destroy(n);
    return rc;
  };
  int rc;
  const int O = dims[n_dims - 1];
  if ((rc = malloc_into(n, &n->theta, o)) || (rc = malloc_into(n, &n->m, o)) || (rc = malloc_into(n, &n->v, o)) ||
      (rc = malloc_into(n, &n->grad, o)) || (rc = malloc_into(n, &n->wbf, o)) || (rc = malloc_into(n, &n->mean, O)) ||
      (rc = malloc_into(n, &n->stdv, O)) || (rc = malloc_into(n, &n->dZa, (size_t)max_batch * wmax)) ||
      (rc = malloc_into(n, &n->dZb, (size_t)max_batch * wmax)) ||
      (rc = malloc_into(n, &n->xb, (size_t)max_batch * dims[0])) || (rc = malloc_into(n, &n->tb, (size_t)max_batch * O)) ||
      (rc = malloc_into(n, &n->partial, kMaxPartials)) ||
      (rc = malloc_into(n, &n->loss, 1)))
    return cleanup(rc);
  {
    int inmax = 0;
    for (int l = 0; l < n->layers; ++l) inmax = std::max(inmax, dims[l]);
    n->ws_floats = (long)kSplitSlices * max_batch * inmax;
    if ((rc = malloc_into(n, &n->ws, (size_t)n->ws_floats))) return cleanup(rc);
  }
  n->Z.resize(n->layers, nullptr);
  n->A.resize(n->layers, nullptr);
  for (int l = 0; l < n->layers; ++l) {
    if ((rc = malloc_into(n, &n->Z[l], (size_t)max_batch * dims[l + 1]))) return cleanup(rc);
    if (l < n->layers - 1 && (rc = malloc_into(n, &n->A[l], (size_t)max_batch * dims[l + 1]))) return cleanup(rc);
  }
  std::vector<float> ones(O, 1.0f);
  hipStream_t s = n->stream;
  if ((rc = hip_rc(hipMemsetAsync(n->m, 0, sizeof(float) * o, s), "zero moments")) ||
      (rc = hip_rc(hipMemsetAsync(n->v, 0, sizeof(float) * o, s), "zero moments")) ||
      (rc = hip_rc(hipMemsetAsync(n->mean, 0, sizeof(float) * O, s), "normalisation")) ||
      (rc = hip_rc(hipMemcpyAsync(n->stdv, ones.data(), sizeof(float) * O, hipMemcpyHostToDevice, s), "normalisation")))
    return cleanup(rc);
  if (params) {
    if ((rc = vemb_mlp_set_params(n, params))) return cleanup(rc);
  } else {
    if ((rc = hip_rc(hipMemsetAsync(n->theta, 0, sizeof(float) * o, s), "zero params")) ||
        (rc = hip_rc(launch_to_bf16(n->theta, n->wbf, o, s), "bf16 copy")))
      return cleanup(rc);
  }
  if ((rc = hip_rc(hipStreamSynchronize(s), "network setup"))) return cleanup(rc);
  *out = n;
  return VEMB_OK;
}

int vemb_mlp_num_params(const vemb_mlp* n, int64_t* count) {
  if (!n || !count) return fail(VEMB_E_INVALID, "NULL argument");
  *count = n->nparams;
  return VEMB_OK;
}

int vemb_mlp_set_params(vemb_mlp* n, const float* params) {
  if (!n || !params) return fail(VEMB_E_INVALID, "NULL argument");
  VEMB_TRY(hip_rc(hipMemcpyAsync(n->theta, params, sizeof(float) * n->nparams, hipMemcpyHostToDevice, n->stream),
                  "parameter upload"));
  VEMB_TRY(hip_rc(launch_to_bf16(n->theta, n->wbf, n->nparams, n->stream), "bf16 copy"));
  return hip_rc(hipStreamSynchronize(n->stream), "parameter upload");
}

int vemb_mlp_get_params(vemb_mlp* n, float* params) {
  if (!n || !params) return fail(VEMB_E_INVALID, "NULL argument");
  VEMB_TRY(hip_rc(hipMemcpyAsync(params, n->theta, sizeof(float) * n->nparams, hipMemcpyDeviceToHost, n->stream),
                  "parameter download"));
  return hip_rc(hipStreamSynchronize(n->stream), "parameter download");
}

int vemb_mlp_fit_normalization(vemb_mlp* n, const float* targets, int count, float rel_floor) {
  if (!n || !targets || count <= 0 || !(rel_floor >= 0.0f))
    return fail(VEMB_E_INVALID, "bad arguments to vemb_mlp_fit_normalization");
  return hip_rc(launch_colstats(targets, count, n->dims.back(), n->mean, n->stdv, kStdFloor, rel_floor, n->stream),
                "normalisation statistics");
}

int vemb_mlp_get_normalization(vemb_mlp* n, float* mean, float* stdv) {
  if (!n || !mean || !stdv) return fail(VEMB_E_INVALID, "NULL argument");
  const int O = n->dims.back();
  VEMB_TRY(hip_rc(hipMemcpyAsync(mean, n->mean, sizeof(float) * O, hipMemcpyDeviceToHost, n->stream), "copy"));
  VEMB_TRY(hip_rc(hipMemcpyAsync(stdv, n->stdv, sizeof(float) * O, hipMemcpyDeviceToHost, n->stream), "copy"));
  return hip_rc(hipStreamSynchronize(n->stream), "normalisation download");
}

int vemb_mlp_set_normalization(vemb_mlp* n, const float* mean, const float* stdv) {
  if (!n || !mean || !stdv) return fail(VEMB_E_INVALID, "NULL argument");
  const int O = n->dims.back();
  for (int j = 0; j < O; ++j)
    if (!(stdv[j] > 0.0f) || !std::isfinite(mean[j])) return fail(VEMB_E_INVALID, "std must be positive, mean finite");
  VEMB_TRY(hip_rc(hipMemcpyAsync(n->mean, mean, sizeof(float) * O, hipMemcpyHostToDevice, n->stream), "copy"));
  VEMB_TRY(hip_rc(hipMemcpyAsync(n->stdv, stdv, sizeof(float) * O, hipMemcpyHostToDevice, n->stream), "copy"));
  return hip_rc(hipStreamSynchronize(n->stream), "normalisation upload");
}

int vemb_mlp_forward(vemb_mlp* n, const float* x, float* y, int batch) {
  if (!n || !x || !y) return fail(VEMB_E_INVALID, "NULL argument");
  VEMB_TRY(check_batch(n, batch));
  VEMB_TRY(forward_pass(n, x, batch));
  return hip_rc(launch_denorm(n->Z[n->layers - 1], n->mean, n->stdv, batch, n->dims.back(), y, n->stream),
                "network output");
}

int vemb_mlp_gradients(vemb_mlp* n, const float* x, const float* targets, int batch, double* loss, float* grad) {
  if (!n || !x || !targets) return fail(VEMB_E_INVALID, "NULL argument");
  VEMB_TRY(check_batch(n, batch));
  VEMB_TRY(backward_pass(n, x, targets, batch));
  if (grad)
    VEMB_TRY(hip_rc(hipMemcpyAsync(grad, n->grad, sizeof(float) * n->nparams, hipMemcpyDeviceToDevice, n->stream),
                    "gradient copy"));
  return read_loss(n, loss);
}

int vemb_mlp_adam_step(vemb_mlp* n, float lr) {
  if (!n || !(lr > 0.0f)) return fail(VEMB_E_INVALID, "bad arguments to vemb_mlp_adam_step");
  ++n->t;
  const double c1 = 1.0 / (1.0 - std::pow((double)kAdamB1, (double)n->t));
  const double c2 = 1.0 / (1.0 - std::pow((double)kAdamB2, (double)n->t));
  return hip_rc(launch_adam(n->theta, n->m, n->v, n->grad, n->wbf, n->nparams, lr, (float)c1, (float)c2, n->stream),
                "Adam step");
}

int vemb_mlp_train_step(vemb_mlp* n, const float* X, const float* T, int count, const int32_t* rows, int batch,
                        float lr, double* loss) {
  if (!n || !X || !T) return fail(VEMB_E_INVALID, "NULL argument");
  VEMB_TRY(check_batch(n, batch));
  if (count <= 0 || (!rows && batch > count)) return fail(VEMB_E_INVALID, "batch exceeds the training set");
  const float* xb = X;
  const float* tb = T;
  if (rows) {
    VEMB_TRY(hip_rc(launch_gather_rows(X, count, rows, batch, n->dims[0], n->xb, n->stream), "gather inputs"));
    VEMB_TRY(hip_rc(launch_gather_rows(T, count, rows, batch, n->dims.back(), n->tb, n->stream), "gather targets"));
    xb = n->xb;
    tb = n->tb;
  }
  VEMB_TRY(backward_pass(n, xb, tb, batch));
  VEMB_TRY(vemb_mlp_adam_step(n, lr));
  return read_loss(n, loss);
}

void vemb_mlp_destroy(vemb_mlp* n) {
  if (!n) return;
  if (n->stream) hipStreamSynchronize(n->stream);
  else hipDeviceSynchronize();
  n->mem.release();
  delete n;
  object_destroyed();
}

}  // extern "C"

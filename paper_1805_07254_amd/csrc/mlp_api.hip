// C-ABI host side of the learned predictor (declared in include/rtc_mlp.h).
//
// Device buffers of a network (float32 unless noted), for max_batch rows:
//   params  W1 [n_hid][n_in], b1 [n_hid], W2 [n_out][n_hid], b2 [n_out]; bfloat16 copies of W1, W2
//   adam    first and second moments of every parameter
//   grads   as the parameters
//   work    Z1 [B][n_hid], H (bfloat16) [B][n_hid], Y [B][n_out], dY [B][n_out] (+ bfloat16),
//           dH [B][n_hid], dZ1 [B][n_hid] (+ bfloat16), per-row squared errors [B]
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "../../include/rtc_mlp.h"
#include "mlp_kernels.h"
#include "rtc_ctx.h"

namespace {

struct Tensor {
  float *p = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
  uint16_t *b = nullptr;   // bfloat16 copy (weights only)
  int64_t n = 0;
};

thread_local std::string g_mlp_err = "no error";

struct DevScope {
  int prev = -1;
  hipError_t status = hipSuccess;
  explicit DevScope(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    status = hipSetDevice(dev);
  }
  ~DevScope() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

template <typename T>
void dfree(T *&p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

bool all_finite(const float *x, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(x[i])) return false;
  return true;
}

}  // namespace

struct rtc_mlp {
  int32_t n_in = 0, n_hid = 0, n_out = 0, max_batch = 0, device = 0;
  Tensor W1, b1, W2, b2;
  float *Z1 = nullptr, *Y = nullptr, *dY = nullptr, *dH = nullptr, *dZ1 = nullptr, *row_sq = nullptr;
  uint16_t *Hb = nullptr, *dYb = nullptr, *dZ1b = nullptr;
  uint16_t *Xb = nullptr;  // a training batch's inputs rounded to bfloat16 once, for both products that read them
  float *ws = nullptr;     // split-K partial tiles of the training products
  int64_t ws_len = 0;
  std::string err = "no error";
};

struct rtc_pred {
  rtc_mlp *net = nullptr;
  int32_t history = 0, n_modes = 0, n_slopes = 0, n_act = 0, frames = 0;   // frames seen, up to history
  int32_t pos = 0;           // ring slot of the next change (hist holds 2 history slots)
  float inv_gain = 1.0f;
  // P [n_modes][ldp], PD [n_modes][ldd], PT [n_slopes][ldt]: rows zero-padded to a multiple of 4
  int64_t ldp = 0, ldd = 0, ldt = 0;
  float *P = nullptr, *PT = nullptr, *PD = nullptr, *mean = nullptr, *std_ = nullptr, *inv_std = nullptr;
  float *hist = nullptr, *m = nullptr, *m_prev = nullptr, *d = nullptr;
  float *s_pred = nullptr;   // [round_up(n_slopes, 16)] feed-forward slopes of predictive frame batches, zero-padded
  int32_t last_mode = RTC_FRAMES_PER_LAUNCH;   // frame mode of the last predictive batch
  std::string err = "no error";
};

namespace {

rtc_status mfail(rtc_mlp *m, rtc_status s, const std::string &msg) {
  if (m) m->err = msg; else g_mlp_err = msg;
  return s;
}

rtc_status hfail(rtc_mlp *m, hipError_t e, const char *what) {
  return mfail(m, e == hipErrorOutOfMemory ? RTC_E_NOMEM : RTC_E_DEVICE,
               std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")");
}

hipError_t alloc_tensor(Tensor &t, int64_t n, bool with_bf16) {
  t.n = n;
  hipError_t e;
  const size_t bytes = (size_t)n * sizeof(float);
  if ((e = hipMalloc(&t.p, bytes)) != hipSuccess || (e = hipMalloc(&t.m, bytes)) != hipSuccess ||
      (e = hipMalloc(&t.v, bytes)) != hipSuccess || (e = hipMalloc(&t.g, bytes)) != hipSuccess)
    return e;
  if (with_bf16 && (e = hipMalloc(&t.b, (size_t)n * sizeof(uint16_t))) != hipSuccess) return e;
  if ((e = hipMemset(t.p, 0, bytes)) != hipSuccess || (e = hipMemset(t.m, 0, bytes)) != hipSuccess ||
      (e = hipMemset(t.v, 0, bytes)) != hipSuccess || (e = hipMemset(t.g, 0, bytes)) != hipSuccess)
    return e;
  if (with_bf16 && (e = hipMemset(t.b, 0, (size_t)n * sizeof(uint16_t))) != hipSuccess) return e;
  return hipSuccess;
}

void free_tensor(Tensor &t) {
  dfree(t.p);
  dfree(t.m);
  dfree(t.v);
  dfree(t.g);
  dfree(t.b);
}

// Forward into m->Z1 / Hb / y (y has batch rows of n_out); xb (nullable): x
// already rounded to bfloat16.
// defer (nullable): the second product may leave its split sums to the
// caller's consumer (launch_loss_grad), which then reads m->ws instead of y.
hipError_t forward(rtc_mlp *m, int32_t B, const float *x, float *y, hipStream_t st, const uint16_t *xb = nullptr,
                   int *defer = nullptr) {
  rtcm::GemmArgs g{};
  g.ws = m->ws;
  g.ws_len = m->ws_len;
  g.M = B;
  g.N = m->n_hid;
  g.K = m->n_in;
  if (xb)
    g.a_bf16 = xb;
  else
    g.a_f32 = x;
  g.sam = m->n_in;
  g.sak = 1;
  g.b_bf16 = m->W1.b;
  g.sbk = 1;
  g.sbn = m->n_in;
  g.alpha = 1.0f;
  g.bias = m->b1.p;
  g.gelu = 1;
  g.ldc = m->n_hid;
  g.c_pre = m->Z1;
  g.c_bf16 = m->Hb;
  hipError_t e = rtcm::launch_gemm(g, st);
  if (e != hipSuccess) return e;
  rtcm::GemmArgs h{};
  h.ws = m->ws;
  h.ws_len = m->ws_len;
  h.M = B;
  h.N = m->n_out;
  h.K = m->n_hid;
  h.a_bf16 = m->Hb;
  h.sam = m->n_hid;
  h.sak = 1;
  h.b_bf16 = m->W2.b;
  h.sbk = 1;
  h.sbn = m->n_hid;
  h.alpha = 1.0f;
  h.bias = m->b2.p;
  h.ldc = m->n_out;
  h.c_f32 = y;
  return rtcm::launch_gemm(h, st, defer);
}

// Batch-1 forward for the predictor step: two bfloat16 GEMV layers with the
// rounding points of the batched forward.
// Arguments of one predictor step (the hidden activations use the network's
// first batch row of Z1; the second layer rounds them to bfloat16 as it reads
// them).
rtcm::PredStepArgs step_args(rtc_pred *p, const float *s, const float *c_prev, float *s_out, float *modes) {
  rtcm::PredStepArgs a{};
  rtc_mlp *m = p->net;
  a.P = p->P;
  a.ldp = p->ldp;
  a.PD = p->PD;
  a.ldd = p->ldd;
  a.PT = p->PT;
  a.ldt = p->ldt;
  a.s = s;
  a.c = c_prev;
  a.n_slopes = p->n_slopes;
  a.n_act = p->n_act;
  a.n_modes = p->n_modes;
  a.history = p->history;
  a.n_in = m->n_in;
  a.n_hid = m->n_hid;
  a.push = p->frames > 0;
  a.full = p->frames >= p->history;              // `history` changes need history + 1 frames
  a.hist = p->hist;
  a.pos = p->pos;
  a.m = p->m;
  a.m_prev = p->m_prev;
  a.mean = p->mean;
  a.std_ = p->std_;
  a.inv_std = p->inv_std;
  a.W1 = m->W1.b;
  a.b1 = m->b1.p;
  a.W2 = m->W2.b;
  a.b2 = m->b2.p;
  a.h = m->Z1;
  a.d = p->d;
  a.modes_out = modes;
  a.s_out = s_out;
  a.inv_gain = p->inv_gain;
  return a;
}

}  // namespace

extern "C" {

rtc_status rtc_mlp_create(int32_t n_in, int32_t n_hidden, int32_t n_out, int32_t max_batch, int32_t device,
                          rtc_mlp **out) {
  if (!out) return mfail(nullptr, RTC_E_ARG, "rtc_mlp_create: NULL output");
  auto ok = [](int32_t v) { return v >= 1 && v <= (1 << 16); };
  if (!ok(n_in) || !ok(n_hidden) || !ok(n_out) || !ok(max_batch) || device < 0)
    return mfail(nullptr, RTC_E_ARG, "rtc_mlp_create: sizes must be in 1..65536 and device >= 0");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0)
    return mfail(nullptr, RTC_E_DEVICE, "rtc_mlp_create: no HIP device available");
  if (device >= ndev) return mfail(nullptr, RTC_E_DEVICE, "rtc_mlp_create: device ordinal out of range");
  rtc_mlp *m = new (std::nothrow) rtc_mlp();
  if (!m) return mfail(nullptr, RTC_E_NOMEM, "rtc_mlp_create: host allocation failed");
  m->n_in = n_in;
  m->n_hid = n_hidden;
  m->n_out = n_out;
  m->max_batch = max_batch;
  m->device = device;
  DevScope ds(device);
  hipError_t e = ds.status;
  const int64_t B = max_batch;
  if (e == hipSuccess) e = alloc_tensor(m->W1, (int64_t)n_hidden * n_in, true);
  if (e == hipSuccess) e = alloc_tensor(m->b1, n_hidden, false);
  if (e == hipSuccess) e = alloc_tensor(m->W2, (int64_t)n_out * n_hidden, true);
  if (e == hipSuccess) e = alloc_tensor(m->b2, n_out, false);
  if (e == hipSuccess) e = hipMalloc(&m->Z1, (size_t)B * n_hidden * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&m->Hb, (size_t)B * n_hidden * sizeof(uint16_t));
  if (e == hipSuccess) e = hipMalloc(&m->Y, (size_t)B * n_out * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&m->dY, (size_t)B * n_out * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&m->dYb, (size_t)B * n_out * sizeof(uint16_t));
  if (e == hipSuccess) e = hipMalloc(&m->dH, (size_t)B * n_hidden * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&m->dZ1, (size_t)B * n_hidden * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&m->dZ1b, (size_t)B * n_hidden * sizeof(uint16_t));
  if (e == hipSuccess) e = hipMalloc(&m->Xb, (size_t)B * n_in * sizeof(uint16_t));
  if (e == hipSuccess) e = hipMalloc(&m->row_sq, (size_t)B * sizeof(float));
  {
    // up to 8 splits of the largest product's output
    const int64_t mn = std::max(std::max(B * n_hidden, B * (int64_t)n_out),
                                std::max((int64_t)n_out * n_hidden, (int64_t)n_hidden * n_in));
    m->ws_len = 8 * mn;
    if (e == hipSuccess) e = hipMalloc(&m->ws, (size_t)m->ws_len * sizeof(float));
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    const rtc_status s = hfail(nullptr, e, "rtc_mlp_create");
    rtc_mlp_destroy(m);
    return s;
  }
  *out = m;
  return RTC_OK;
}

rtc_status rtc_mlp_set_params(rtc_mlp *m, const float *W1, const float *b1, const float *W2, const float *b2) {
  if (!m) return mfail(nullptr, RTC_E_ARG, "rtc_mlp_set_params: NULL network");
  if (!W1 || !b1 || !W2 || !b2) return mfail(m, RTC_E_ARG, "rtc_mlp_set_params: NULL parameter");
  if (!all_finite(W1, m->W1.n) || !all_finite(b1, m->b1.n) || !all_finite(W2, m->W2.n) || !all_finite(b2, m->b2.n))
    return mfail(m, RTC_E_NONFINITE, "rtc_mlp_set_params: non-finite parameter");
  DevScope ds(m->device);
  hipError_t e = ds.status;
  if (e == hipSuccess) e = hipDeviceSynchronize();
  const float *src[4] = {W1, b1, W2, b2};
  Tensor *dst[4] = {&m->W1, &m->b1, &m->W2, &m->b2};
  for (int i = 0; i < 4 && e == hipSuccess; ++i) {
    Tensor &t = *dst[i];
    const size_t bytes = (size_t)t.n * sizeof(float);
    e = hipMemcpy(t.p, src[i], bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(t.m, 0, bytes);
    if (e == hipSuccess) e = hipMemset(t.v, 0, bytes);
    if (e == hipSuccess && t.b) e = rtcm::launch_round_bf16(t.p, t.b, t.n, nullptr);
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  return e == hipSuccess ? RTC_OK : hfail(m, e, "rtc_mlp_set_params");
}

rtc_status rtc_mlp_get_params(rtc_mlp *m, float *W1, float *b1, float *W2, float *b2) {
  if (!m) return mfail(nullptr, RTC_E_ARG, "rtc_mlp_get_params: NULL network");
  if (!W1 || !b1 || !W2 || !b2) return mfail(m, RTC_E_ARG, "rtc_mlp_get_params: NULL output");
  DevScope ds(m->device);
  hipError_t e = ds.status;
  if (e == hipSuccess) e = hipDeviceSynchronize();
  float *dst[4] = {W1, b1, W2, b2};
  const Tensor *src[4] = {&m->W1, &m->b1, &m->W2, &m->b2};
  for (int i = 0; i < 4 && e == hipSuccess; ++i)
    e = hipMemcpy(dst[i], src[i]->p, (size_t)src[i]->n * sizeof(float), hipMemcpyDeviceToHost);
  return e == hipSuccess ? RTC_OK : hfail(m, e, "rtc_mlp_get_params");
}

rtc_status rtc_mlp_forward(rtc_mlp *m, int32_t batch, const float *d_x, float *d_y, void *hip_stream) {
  if (!m) return mfail(nullptr, RTC_E_ARG, "rtc_mlp_forward: NULL network");
  if (batch < 1 || batch > m->max_batch) return mfail(m, RTC_E_ARG, "rtc_mlp_forward: batch outside 1..max_batch");
  if (!d_x || !d_y) return mfail(m, RTC_E_ARG, "rtc_mlp_forward: NULL input or output");
  DevScope ds(m->device);
  if (ds.status != hipSuccess) return hfail(m, ds.status, "rtc_mlp_forward: hipSetDevice");
  const hipError_t e = forward(m, batch, d_x, d_y, static_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? RTC_OK : hfail(m, e, "rtc_mlp_forward");
}

rtc_status rtc_mlp_loss_grad(rtc_mlp *m, int32_t B, const float *d_x, const float *d_t, float *d_loss,
                             void *hip_stream) {
  if (!m) return mfail(nullptr, RTC_E_ARG, "rtc_mlp_loss_grad: NULL network");
  if (B < 1 || B > m->max_batch) return mfail(m, RTC_E_ARG, "rtc_mlp_loss_grad: batch outside 1..max_batch");
  if (!d_x || !d_t || !d_loss) return mfail(m, RTC_E_ARG, "rtc_mlp_loss_grad: NULL argument");
  DevScope ds(m->device);
  if (ds.status != hipSuccess) return hfail(m, ds.status, "rtc_mlp_loss_grad: hipSetDevice");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  // the inputs in bfloat16 once (the products would round them as they load
  // them, once per tile that reads them)
  hipError_t e = rtcm::launch_round_bf16(d_x, m->Xb, (int64_t)B * m->n_in, st);
  // the output layer's split sums (if it splits) are added by the loss kernel
  int defer_y = 0;
  if (e == hipSuccess) e = forward(m, B, d_x, m->Y, st, m->Xb, &defer_y);
  if (e == hipSuccess)
    e = rtcm::launch_loss_grad(m->Y, d_t, B, m->n_out, m->dY, m->dYb, m->row_sq, d_loss, st,
                               defer_y ? m->ws : nullptr, defer_y, m->b2.p);
  if (e == hipSuccess) {                            // dW2 = dY^T H
    rtcm::GemmArgs g{};
    g.ws = m->ws;
    g.ws_len = m->ws_len;
    g.M = m->n_out;
    g.N = m->n_hid;
    g.K = B;
    g.a_bf16 = m->dYb;
    g.sam = 1;
    g.sak = m->n_out;
    g.b_bf16 = m->Hb;
    g.sbk = m->n_hid;
    g.sbn = 1;
    g.alpha = 1.0f;
    g.ldc = m->n_hid;
    g.c_f32 = m->W2.g;
    e = rtcm::launch_gemm(g, st);
  }
  if (e == hipSuccess) e = rtcm::launch_col_sum(m->dY, B, m->n_out, m->b2.g, st);
  int defer_h = 0;
  if (e == hipSuccess) {                            // dH = dY W2
    rtcm::GemmArgs g{};
    g.ws = m->ws;
    g.ws_len = m->ws_len;
    g.M = B;
    g.N = m->n_hid;
    g.K = m->n_out;
    g.a_bf16 = m->dYb;
    g.sam = m->n_out;
    g.sak = 1;
    g.b_bf16 = m->W2.b;
    g.sbk = m->n_hid;
    g.sbn = 1;
    g.alpha = 1.0f;
    g.ldc = m->n_hid;
    g.c_f32 = m->dH;
    e = rtcm::launch_gemm(g, st, &defer_h);           // split sums added by the GELU derivative kernel
  }
  if (e == hipSuccess)
    e = rtcm::launch_gelu_back(m->dH, m->Z1, m->dZ1, m->dZ1b, (int64_t)B * m->n_hid, st,
                               defer_h ? m->ws : nullptr, defer_h);
  if (e == hipSuccess) {                            // dW1 = dZ1^T X
    rtcm::GemmArgs g{};
    g.ws = m->ws;
    g.ws_len = m->ws_len;
    g.M = m->n_hid;
    g.N = m->n_in;
    g.K = B;
    g.a_bf16 = m->dZ1b;
    g.sam = 1;
    g.sak = m->n_hid;
    g.b_bf16 = m->Xb;
    g.sbk = m->n_in;
    g.sbn = 1;
    g.alpha = 1.0f;
    g.ldc = m->n_in;
    g.c_f32 = m->W1.g;
    e = rtcm::launch_gemm(g, st);
  }
  if (e == hipSuccess) e = rtcm::launch_col_sum(m->dZ1, B, m->n_hid, m->b1.g, st);
  return e == hipSuccess ? RTC_OK : hfail(m, e, "rtc_mlp_loss_grad");
}

rtc_status rtc_mlp_get_grads(rtc_mlp *m, float *dW1, float *db1, float *dW2, float *db2) {
  if (!m) return mfail(nullptr, RTC_E_ARG, "rtc_mlp_get_grads: NULL network");
  if (!dW1 || !db1 || !dW2 || !db2) return mfail(m, RTC_E_ARG, "rtc_mlp_get_grads: NULL output");
  DevScope ds(m->device);
  hipError_t e = ds.status;
  if (e == hipSuccess) e = hipDeviceSynchronize();
  float *dst[4] = {dW1, db1, dW2, db2};
  const Tensor *src[4] = {&m->W1, &m->b1, &m->W2, &m->b2};
  for (int i = 0; i < 4 && e == hipSuccess; ++i)
    e = hipMemcpy(dst[i], src[i]->g, (size_t)src[i]->n * sizeof(float), hipMemcpyDeviceToHost);
  return e == hipSuccess ? RTC_OK : hfail(m, e, "rtc_mlp_get_grads");
}

rtc_status rtc_mlp_adam(rtc_mlp *m, float lr, float beta1, float beta2, float eps, int32_t step, void *hip_stream) {
  if (!m) return mfail(nullptr, RTC_E_ARG, "rtc_mlp_adam: NULL network");
  if (step < 1 || !std::isfinite(lr) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
      !(eps > 0.0f))
    return mfail(m, RTC_E_ARG, "rtc_mlp_adam: need step >= 1, finite lr, betas in [0, 1), eps > 0");
  DevScope ds(m->device);
  if (ds.status != hipSuccess) return hfail(m, ds.status, "rtc_mlp_adam: hipSetDevice");
  const float c1 = (float)(1.0 - std::pow((double)beta1, (double)step));
  const float c2 = (float)(1.0 - std::pow((double)beta2, (double)step));
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  // the four tensors in one launch
  const Tensor *ts[4] = {&m->W1, &m->b1, &m->W2, &m->b2};
  rtcm::AdamTensor at[4];
  for (int i = 0; i < 4; ++i) at[i] = rtcm::AdamTensor{ts[i]->p, ts[i]->m, ts[i]->v, ts[i]->g, ts[i]->b, ts[i]->n};
  const hipError_t e = rtcm::launch_adam_multi(at, 4, lr, beta1, beta2, eps, c1, c2, st);
  return e == hipSuccess ? RTC_OK : hfail(m, e, "rtc_mlp_adam");
}

void rtc_mlp_destroy(rtc_mlp *m) {
  if (!m) return;
  DevScope ds(m->device);
  if (ds.status == hipSuccess) (void)hipDeviceSynchronize();
  free_tensor(m->W1);
  free_tensor(m->b1);
  free_tensor(m->W2);
  free_tensor(m->b2);
  dfree(m->Z1);
  dfree(m->Hb);
  dfree(m->Y);
  dfree(m->dY);
  dfree(m->dYb);
  dfree(m->dH);
  dfree(m->dZ1);
  dfree(m->dZ1b);
  dfree(m->Xb);
  dfree(m->ws);
  dfree(m->row_sq);
  delete m;
}

// ---------------------------------------------------------------------------
// predictor
static rtc_status pfail(rtc_pred *p, rtc_status s, const std::string &msg) {
  if (p) p->err = msg; else g_mlp_err = msg;
  return s;
}

void rtc_pred_destroy(rtc_pred *p);

rtc_status rtc_pred_create(rtc_mlp *net, int32_t history, int32_t n_modes, int32_t n_slopes, int32_t n_act,
                           const float *P, const float *PD, const float *mean, const float *std_, float gain,
                           rtc_pred **out) {
  if (!net || !out) return pfail(nullptr, RTC_E_ARG, "rtc_pred_create: NULL network or output");
  if (history < 1 || n_modes < 1 || n_slopes < 1 || n_act < 1)
    return pfail(nullptr, RTC_E_ARG, "rtc_pred_create: sizes must be >= 1");
  if ((int64_t)history * n_modes != net->n_in || n_modes != net->n_out)
    return pfail(nullptr, RTC_E_ARG, "rtc_pred_create: the network must map history * n_modes inputs to n_modes");
  if (!P || !PD || !mean || !std_) return pfail(nullptr, RTC_E_ARG, "rtc_pred_create: NULL matrix");
  if (!all_finite(P, (int64_t)n_modes * n_slopes) || !all_finite(PD, (int64_t)n_modes * n_act) ||
      !all_finite(mean, n_modes) || !all_finite(std_, n_modes) || !std::isfinite(gain) || !(gain > 0.0f))
    return pfail(nullptr, RTC_E_NONFINITE, "rtc_pred_create: non-finite input or non-positive gain");
  const int64_t ldp = (n_slopes + 3) / 4 * 4, ldd = (n_act + 3) / 4 * 4, ldt = (n_modes + 3) / 4 * 4;
  std::vector<float> inv((size_t)n_modes), Pp((size_t)n_modes * ldp, 0.0f), PDp((size_t)n_modes * ldd, 0.0f),
      PT((size_t)n_slopes * ldt, 0.0f);
  for (int32_t j = 0; j < n_modes; ++j) {
    if (!(std_[j] > 0.0f)) return pfail(nullptr, RTC_E_NONFINITE, "rtc_pred_create: std must be positive");
    inv[(size_t)j] = 1.0f / std_[j];
    for (int32_t i = 0; i < n_slopes; ++i) {
      Pp[(size_t)j * ldp + i] = P[(size_t)j * n_slopes + i];
      PT[(size_t)i * ldt + j] = P[(size_t)j * n_slopes + i];
    }
    for (int32_t i = 0; i < n_act; ++i) PDp[(size_t)j * ldd + i] = PD[(size_t)j * n_act + i];
  }
  rtc_pred *p = new (std::nothrow) rtc_pred();
  if (!p) return pfail(nullptr, RTC_E_NOMEM, "rtc_pred_create: host allocation failed");
  p->net = net;
  p->history = history;
  p->n_modes = n_modes;
  p->n_slopes = n_slopes;
  p->n_act = n_act;
  p->inv_gain = 1.0f / gain;
  p->ldp = ldp;
  p->ldd = ldd;
  p->ldt = ldt;
  DevScope ds(net->device);
  hipError_t e = ds.status;
  const size_t fm = sizeof(float) * (size_t)n_modes;
  const size_t s_pad = sizeof(float) * (size_t)((n_slopes + 15) / 16 * 16);
  if (e == hipSuccess) e = hipMalloc(&p->P, sizeof(float) * Pp.size());
  if (e == hipSuccess) e = hipMalloc(&p->PT, sizeof(float) * PT.size());
  if (e == hipSuccess) e = hipMalloc(&p->PD, sizeof(float) * PDp.size());
  if (e == hipSuccess) e = hipMalloc(&p->mean, fm);
  if (e == hipSuccess) e = hipMalloc(&p->std_, fm);
  if (e == hipSuccess) e = hipMalloc(&p->inv_std, fm);
  if (e == hipSuccess) e = hipMalloc(&p->hist, fm * 2 * history);
  if (e == hipSuccess) e = hipMalloc(&p->m, fm);
  if (e == hipSuccess) e = hipMalloc(&p->m_prev, fm);
  if (e == hipSuccess) e = hipMalloc(&p->d, fm);
  if (e == hipSuccess) e = hipMalloc(&p->s_pred, s_pad);
  if (e == hipSuccess) e = hipMemcpy(p->P, Pp.data(), sizeof(float) * Pp.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->PT, PT.data(), sizeof(float) * PT.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->PD, PDp.data(), sizeof(float) * PDp.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->mean, mean, fm, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->std_, std_, fm, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->inv_std, inv.data(), fm, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(p->hist, 0, fm * 2 * history);
  if (e == hipSuccess) e = hipMemset(p->s_pred, 0, s_pad);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    const rtc_status s = pfail(nullptr, e == hipErrorOutOfMemory ? RTC_E_NOMEM : RTC_E_DEVICE,
                               std::string("rtc_pred_create: ") + hipGetErrorName(e));
    rtc_pred_destroy(p);
    return s;
  }
  *out = p;
  return RTC_OK;
}

rtc_status rtc_pred_reset(rtc_pred *p) {
  if (!p) return pfail(nullptr, RTC_E_ARG, "rtc_pred_reset: NULL predictor");
  DevScope ds(p->net->device);
  hipError_t e = ds.status;
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemset(p->hist, 0, sizeof(float) * (size_t)p->n_modes * 2 * p->history);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) return pfail(p, RTC_E_DEVICE, std::string("rtc_pred_reset: ") + hipGetErrorName(e));
  p->frames = 0;
  p->pos = 0;
  return RTC_OK;
}

// After a step: the ring moves on when the step stored a change.
static void advance(rtc_pred *p) {
  if (p->frames > 0) p->pos = (p->pos + 1) % p->history;
  if (p->frames < p->history) ++p->frames;
}

rtc_status rtc_pred_step(rtc_pred *p, const float *d_slopes, const float *d_cmd_prev, float *d_slopes_out,
                         float *d_modes, void *hip_stream) {
  if (!p) return pfail(nullptr, RTC_E_ARG, "rtc_pred_step: NULL predictor");
  if (!d_slopes || !d_cmd_prev || !d_slopes_out) return pfail(p, RTC_E_ARG, "rtc_pred_step: NULL argument");
  if (d_slopes_out == d_slopes || d_slopes_out == d_cmd_prev)
    return pfail(p, RTC_E_ARG, "rtc_pred_step: d_slopes_out aliases an input");
  DevScope ds(p->net->device);
  if (ds.status != hipSuccess) return pfail(p, RTC_E_DEVICE, "rtc_pred_step: hipSetDevice");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const hipError_t e = rtcm::launch_pred_step(step_args(p, d_slopes, d_cmd_prev, d_slopes_out, d_modes), st);
  if (e != hipSuccess) return pfail(p, RTC_E_DEVICE, std::string("rtc_pred_step: ") + hipGetErrorName(e));
  advance(p);
  return RTC_OK;
}

// Predictor step of a predictive frame: the feed-forward slopes go to the
// predictor's own padded buffer, which the reconstruction then multiplies.
static hipError_t pred_frame_step(void *arg, const float *s, const float *c_prev, const float **s_use,
                                  hipStream_t st) {
  rtc_pred *p = static_cast<rtc_pred *>(arg);
  const hipError_t e = rtcm::launch_pred_step(step_args(p, s, c_prev, p->s_pred, nullptr), st);
  if (e == hipSuccess) advance(p);
  *s_use = p->s_pred;
  return e;
}

rtc_status rtc_pred_frame_batch(rtc_ctx *c, rtc_pred *p, int32_t n_frames, const uint16_t *d_pixels,
                                int64_t frame_stride, float *d_cmd, float *d_slopes, uint64_t *d_ts,
                                void *hip_stream) {
  if (!c || !p) return pfail(p, RTC_E_ARG, "rtc_pred_frame_batch: NULL context or predictor");
  if (p->n_slopes != c->n_slopes || p->n_act != c->n_act)
    return pfail(p, RTC_E_ARG, "rtc_pred_frame_batch: predictor and context sizes differ");
  if (p->net->device != c->device) return pfail(p, RTC_E_ARG, "rtc_pred_frame_batch: different devices");
  if (!c->calib_loaded || !c->cmat_loaded)
    return pfail(p, RTC_E_STATE, "rtc_pred_frame_batch: load the context's calibration and control matrix first");
  if (c->state_invalid) return pfail(p, RTC_E_STATE, "rtc_pred_frame_batch: " STATE_INVALID_MSG);
  if (n_frames < 0) return pfail(p, RTC_E_ARG, "rtc_pred_frame_batch: n_frames < 0");
  if (n_frames == 0) return RTC_OK;
  if (!d_pixels || !d_cmd) return pfail(p, RTC_E_ARG, "rtc_pred_frame_batch: NULL pixels or cmd");
  if (frame_stride < c->frame_elems)
    return pfail(p, RTC_E_ARG, "rtc_pred_frame_batch: frame_stride shorter than a frame");
  DevScope ds(c->device);
  if (ds.status != hipSuccess) return pfail(p, RTC_E_DEVICE, "rtc_pred_frame_batch: hipSetDevice");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  // persistent mode: every frame in one launch when the built kernels cover
  // the shape (8-byte weight loads need rows of a multiple of 4 elements)
  const rtc_mlp *m = p->net;
  const bool vec = m->n_in % 4 == 0 && m->n_hid % 4 == 0 && reinterpret_cast<uintptr_t>(m->W1.b) % 8 == 0 &&
                   reinterpret_cast<uintptr_t>(m->W2.b) % 8 == 0;
  if (vec) {
    bool ran = false;
    const rtc_status s = rtcx::enqueue_pred_frames(c, step_args(p, nullptr, nullptr, nullptr, nullptr), p->frames,
                                                   n_frames, d_pixels, frame_stride, d_cmd, d_slopes, d_ts, st,
                                                   "rtc_pred_frame_batch: persistent launch", &ran);
    if (s != RTC_OK) return pfail(p, s, c->err);
    if (ran) {
      for (int32_t f = 0; f < n_frames; ++f) advance(p);
      p->last_mode = RTC_FRAMES_PERSISTENT;
      return RTC_OK;
    }
  }
  for (int32_t f = 0; f < n_frames; ++f) {
    const rtc_status s = rtcx::enqueue_frame_with(
        c, d_pixels + (int64_t)f * frame_stride, d_cmd + (int64_t)f * c->n_act,
        d_slopes ? d_slopes + (int64_t)f * c->n_slopes : nullptr, nullptr, nullptr,
        d_ts ? d_ts + 2 * (int64_t)f : nullptr, st, "rtc_pred_frame_batch: launch", pred_frame_step, p);
    if (s != RTC_OK) return pfail(p, s, c->err);
  }
  p->last_mode = RTC_FRAMES_PER_LAUNCH;
  return RTC_OK;
}

rtc_status rtc_pred_last_batch_mode(const rtc_pred *p, int32_t *mode) {
  if (!p || !mode) return pfail(nullptr, RTC_E_ARG, "rtc_pred_last_batch_mode: NULL argument");
  *mode = p->last_mode;
  return RTC_OK;
}

void rtc_pred_destroy(rtc_pred *p) {
  if (!p) return;
  DevScope ds(p->net ? p->net->device : 0);
  if (ds.status == hipSuccess) (void)hipDeviceSynchronize();
  dfree(p->P);
  dfree(p->PT);
  dfree(p->PD);
  dfree(p->mean);
  dfree(p->std_);
  dfree(p->inv_std);
  dfree(p->hist);
  dfree(p->m);
  dfree(p->m_prev);
  dfree(p->d);
  dfree(p->s_pred);
  delete p;
}

const char *rtc_mlp_error_string(const rtc_mlp *m) { return m ? m->err.c_str() : g_mlp_err.c_str(); }
const char *rtc_pred_error_string(const rtc_pred *p) { return p ? p->err.c_str() : g_mlp_err.c_str(); }

}  // extern "C"

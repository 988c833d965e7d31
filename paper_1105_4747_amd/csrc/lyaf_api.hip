// lyaf_api.hip -- the C ABI declared in include/lyaf.h: host-side validation,
// per-(device, stream) workspaces, work lists, and the kernel launches.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "lyaf_internal.h"

namespace lyaf {
namespace {

std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, Workspace *> g_ws;

// Host mirrors of the work list currently uploaded to a workspace.
struct HostPlan {
  std::vector<int64_t> offsets;    // [S+1]
  std::vector<int64_t> item_base;  // [S+1]
  int64_t n_items = 0;
  // pinned staging
  int64_t *h_off = nullptr;
  int2 *h_items = nullptr;
  int64_t *h_ib = nullptr;
  int64_t h_off_cap = 0, h_items_cap = 0, h_ib_cap = 0;
};
std::map<Workspace *, HostPlan> g_plans;

int map_err(hipError_t e) {
  if (e == hipSuccess) return LYAF_OK;
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return LYAF_ENOMEM;
  return LYAF_EDEVICE;
}

template <typename T>
hipError_t grow_dev(T *&p, int64_t &cap, int64_t need) {
  if (need <= cap) return hipSuccess;
  if (p) {
    hipError_t e = hipFree(p);
    if (e != hipSuccess) return e;
    p = nullptr;
    cap = 0;
  }
  const int64_t n = std::max<int64_t>(need, 64);
  hipError_t e = hipMalloc((void **)&p, (size_t)n * sizeof(T));
  if (e != hipSuccess) return e;
  cap = n;
  return hipSuccess;
}

template <typename T>
hipError_t grow_host(T *&p, int64_t &cap, int64_t need) {
  if (need <= cap) return hipSuccess;
  if (p) {
    hipError_t e = hipHostFree(p);
    if (e != hipSuccess) return e;
    p = nullptr;
    cap = 0;
  }
  const int64_t n = std::max<int64_t>(need, 64);
  hipError_t e = hipHostMalloc((void **)&p, (size_t)n * sizeof(T), hipHostMallocDefault);
  if (e != hipSuccess) return e;
  cap = n;
  return hipSuccess;
}

// Workspace of the current device for `st` (created on first use).
int get_ws(hipStream_t st, Workspace **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return map_err(e);
  auto key = std::make_pair(dev, st);
  auto it = g_ws.find(key);
  if (it != g_ws.end()) {
    *out = it->second;
    return LYAF_OK;
  }
  Workspace *w = new Workspace();
  w->device = dev;
  w->stream = st;
  if ((e = hipMalloc((void **)&w->status, sizeof(uint32_t))) != hipSuccess ||
      (e = hipMalloc((void **)&w->partials, sizeof(double) * 4 * kMaxPartialBlocks)) != hipSuccess ||
      (e = hipMalloc((void **)&w->norm, sizeof(NormState))) != hipSuccess ||
      (e = hipMalloc((void **)&w->ratio, sizeof(double))) != hipSuccess ||
      (e = hipMemset(w->status, 0, sizeof(uint32_t))) != hipSuccess ||
      (e = hipMemset(w->norm, 0, sizeof(NormState))) != hipSuccess ||
      (e = hipMemset(w->ratio, 0, sizeof(double))) != hipSuccess) {
    delete w;
    return map_err(e);
  }
  g_ws[key] = w;
  *out = w;
  return LYAF_OK;
}

// Validate skewers and parameters on the host.  Returns LYAF_OK or EINVAL.
int check_args(const lyaf_skewers *sk, const lyaf_params *prm, int64_t *P_out) {
  if (!sk || !prm) return LYAF_EINVAL;
  if (sk->n_skewers < 0) return LYAF_EINVAL;
  if (!(prm->tau_ref > 0.0) || !isfinite(prm->tau_ref)) return LYAF_EINVAL;
  if (!(prm->delta_pivot > 0.0)) return LYAF_EINVAL;  // +INF allowed
  if (!(prm->window_k >= 0.0) || !isfinite(prm->window_k)) return LYAF_EINVAL;
  const int64_t S = sk->n_skewers;
  int64_t P = 0;
  if (S > 0) {
    if (!sk->offsets) return LYAF_EINVAL;
    if (sk->offsets[0] != 0) return LYAF_EINVAL;
    for (int64_t s = 0; s < S; ++s) {
      const int64_t n = sk->offsets[s + 1] - sk->offsets[s];
      // pixel offsets within a skewer are formed exactly in FP32: N <= 2^24
      if (n < 0 || n > (int64_t(1) << 24)) return LYAF_EINVAL;
    }
    P = sk->offsets[S];
    if (P > 0 && (!sk->delta || !sk->vpec)) return LYAF_EINVAL;
    if (!sk->dv || !sk->T0 || !sk->gamma) return LYAF_EINVAL;
  }
  *P_out = P;
  return LYAF_OK;
}

// Upload offsets, the (skewer, tile) work list and the per-skewer first item,
// unless the workspace already holds this exact set of offsets.
int ensure_plan(Workspace *ws, const lyaf_skewers *sk, HostPlan **out) {
  HostPlan &hp = g_plans[ws];
  *out = &hp;
  const int64_t S = sk->n_skewers;
  if ((int64_t)hp.offsets.size() == S + 1 &&
      memcmp(hp.offsets.data(), sk->offsets, sizeof(int64_t) * (size_t)(S + 1)) == 0)
    return LYAF_OK;
  hipError_t e;
  // the pinned staging buffers may still feed an earlier copy on this stream
  if ((e = hipStreamSynchronize(ws->stream)) != hipSuccess) return map_err(e);
  hp.offsets.assign(sk->offsets, sk->offsets + S + 1);
  hp.item_base.assign((size_t)S + 1, 0);
  int64_t ni = 0;
  for (int64_t s = 0; s < S; ++s) {
    hp.item_base[s] = ni;
    ni += (hp.offsets[s + 1] - hp.offsets[s] + kTauTile - 1) / kTauTile;
  }
  hp.item_base[S] = ni;
  hp.n_items = ni;
  if ((e = grow_host(hp.h_off, hp.h_off_cap, S + 1)) != hipSuccess ||
      (e = grow_host(hp.h_ib, hp.h_ib_cap, S + 1)) != hipSuccess ||
      (e = grow_host(hp.h_items, hp.h_items_cap, ni)) != hipSuccess ||
      (e = grow_dev(ws->offsets, ws->off_cap, S + 1)) != hipSuccess ||
      (e = grow_dev(ws->item_base, ws->ib_cap, S + 1)) != hipSuccess ||
      (e = grow_dev(ws->items, ws->items_cap, ni)) != hipSuccess ||
      (e = grow_dev(ws->skc, ws->skc_cap, S)) != hipSuccess) {
    hp.offsets.clear();
    return map_err(e);
  }
  memcpy(hp.h_off, hp.offsets.data(), sizeof(int64_t) * (size_t)(S + 1));
  memcpy(hp.h_ib, hp.item_base.data(), sizeof(int64_t) * (size_t)(S + 1));
  for (int64_t s = 0; s < S; ++s) {
    const int64_t nt = hp.item_base[s + 1] - hp.item_base[s];
    for (int64_t t = 0; t < nt; ++t)
      hp.h_items[hp.item_base[s] + t] = make_int2((int)s, (int)t);
  }
  if ((e = hipMemcpyAsync(ws->offsets, hp.h_off, sizeof(int64_t) * (size_t)(S + 1),
                          hipMemcpyHostToDevice, ws->stream)) != hipSuccess ||
      (e = hipMemcpyAsync(ws->item_base, hp.h_ib, sizeof(int64_t) * (size_t)(S + 1),
                          hipMemcpyHostToDevice, ws->stream)) != hipSuccess ||
      (ni > 0 && (e = hipMemcpyAsync(ws->items, hp.h_items, sizeof(int2) * (size_t)ni,
                                     hipMemcpyHostToDevice, ws->stream)) != hipSuccess)) {
    hp.offsets.clear();
    return map_err(e);
  }
  return LYAF_OK;
}

Batch make_batch(const lyaf_skewers *sk, const lyaf_params *prm, Workspace *ws) {
  Batch b;
  b.delta = sk->delta;
  b.vpec = sk->vpec;
  b.dv = sk->dv;
  b.T0 = sk->T0;
  b.gamma = sk->gamma;
  b.offsets = ws->offsets;
  b.skc = ws->skc;
  b.n_skewers = sk->n_skewers;
  b.tau_ref = (float)prm->tau_ref;
  b.pivot = isinf(prm->delta_pivot) ? INFINITY : (float)prm->delta_pivot;
  b.window_k = (float)prm->window_k;
  b.status = ws->status;
  return b;
}

}  // namespace
}  // namespace lyaf

using namespace lyaf;

extern "C" {

int lyaf_version(void) { return 100; }

const char *lyaf_strerror(int code) {
  switch (code) {
    case LYAF_OK: return "ok";
    case LYAF_EINVAL: return "invalid argument";
    case LYAF_EDOMAIN: return "value outside the model domain";
    case LYAF_ENOROOT: return "no mean-flux root exists";
    case LYAF_ENOCONV: return "mean-flux root-find did not converge";
    case LYAF_EDEVICE: return "HIP runtime error";
    case LYAF_ENOMEM: return "device memory allocation failed";
    default: return "unknown error";
  }
}

int lyaf_tau(const lyaf_skewers *sk, const lyaf_params *prm, float *tau_out, void *stream) {
  int64_t P = 0;
  int rc = check_args(sk, prm, &P);
  if (rc) return rc;
  if (P > 0 && !tau_out) return LYAF_EINVAL;
  if (P == 0) return LYAF_OK;
  std::lock_guard<std::mutex> lk(g_mu);
  hipStream_t st = (hipStream_t)stream;
  Workspace *ws = nullptr;
  if ((rc = get_ws(st, &ws))) return rc;
  HostPlan *hp = nullptr;
  if ((rc = ensure_plan(ws, sk, &hp))) return rc;
  const Batch b = make_batch(sk, prm, ws);
  hipError_t e = launch_reach(b, st);
  if (e != hipSuccess) return map_err(e);
  const int64_t S = sk->n_skewers;
  if (prm->flags & LYAF_FLAG_PLAIN) {
    for (int64_t s = 0; s < S && e == hipSuccess; ++s)
      e = launch_tau_plain(b, s, hp->offsets[s + 1] - hp->offsets[s], tau_out, st);
  } else if (prm->flags & LYAF_FLAG_PER_SKEWER) {
    for (int64_t s = 0; s < S && e == hipSuccess; ++s)
      e = launch_tau_window(b, ws->items + hp->item_base[s],
                            hp->item_base[s + 1] - hp->item_base[s], tau_out, st);
  } else {
    e = launch_tau_window(b, ws->items, hp->n_items, tau_out, st);
  }
  return map_err(e);
}

int lyaf_normalise_mean_flux(int64_t n_pix, float *tau_inout, float *F_out, double target_F,
                             double *A_dev, void *stream) {
  if (n_pix <= 0 || !tau_inout || !A_dev) return LYAF_EINVAL;
  if (!(target_F > 0.0 && target_F < 1.0)) return LYAF_EINVAL;
  if (F_out == tau_inout) return LYAF_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  hipStream_t st = (hipStream_t)stream;
  Workspace *ws = nullptr;
  int rc = get_ws(st, &ws);
  if (rc) return rc;
  return map_err(launch_norm(n_pix, tau_inout, F_out, target_F, A_dev, *ws, st));
}

int lyaf_normalise_mean_flux_backward(int64_t n_pix, const float *tau_raw, const double *A_dev,
                                      const float *grad_F, const float *grad_tau_scaled,
                                      int implicit_A, float *grad_tau_raw_out, void *stream) {
  if (n_pix < 0) return LYAF_EINVAL;
  if (n_pix == 0) return LYAF_OK;
  if (!tau_raw || !A_dev || !grad_tau_raw_out) return LYAF_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  hipStream_t st = (hipStream_t)stream;
  Workspace *ws = nullptr;
  int rc = get_ws(st, &ws);
  if (rc) return rc;
  return map_err(launch_norm_backward(n_pix, tau_raw, A_dev, grad_F, grad_tau_scaled,
                                      implicit_A ? 1 : 0, grad_tau_raw_out, *ws, st));
}

int lyaf_tau_backward(const lyaf_skewers *sk, const lyaf_params *prm, const float *grad_tau_raw,
                      float *grad_delta, float *grad_vpec, double *grad_T0, double *grad_gamma,
                      void *stream) {
  int64_t P = 0;
  int rc = check_args(sk, prm, &P);
  if (rc) return rc;
  if (P > 0 && (!grad_tau_raw || !grad_delta || !grad_vpec)) return LYAF_EINVAL;
  if (sk->n_skewers == 0) return LYAF_OK;
  std::lock_guard<std::mutex> lk(g_mu);
  hipStream_t st = (hipStream_t)stream;
  Workspace *ws = nullptr;
  if ((rc = get_ws(st, &ws))) return rc;
  HostPlan *hp = nullptr;
  if ((rc = ensure_plan(ws, sk, &hp))) return rc;
  hipError_t e = grow_dev(ws->gpart, ws->gpart_cap, 2 * std::max<int64_t>(hp->n_items, 1));
  if (e != hipSuccess) return map_err(e);
  const Batch b = make_batch(sk, prm, ws);
  if ((e = launch_reach(b, st)) != hipSuccess) return map_err(e);
  if (hp->n_items == 0) {
    // every skewer is empty: the per-skewer sums are zero
    if (grad_T0 && (e = hipMemsetAsync(grad_T0, 0, sizeof(double) * (size_t)sk->n_skewers, st)))
      return map_err(e);
    if (grad_gamma &&
        (e = hipMemsetAsync(grad_gamma, 0, sizeof(double) * (size_t)sk->n_skewers, st)))
      return map_err(e);
    return LYAF_OK;
  }
  return map_err(launch_tau_adjoint(b, ws->items, hp->n_items, ws->item_base, grad_tau_raw,
                                    grad_delta, grad_vpec, grad_T0, grad_gamma, ws->gpart, st));
}

int lyaf_status_read(void *stream, uint32_t *device_status) {
  if (!device_status) return LYAF_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  hipStream_t st = (hipStream_t)stream;
  Workspace *ws = nullptr;
  int rc = get_ws(st, &ws);
  if (rc) return rc;
  uint32_t v = 0;
  hipError_t e;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return map_err(e);
  if ((e = hipMemcpy(&v, ws->status, sizeof(uint32_t), hipMemcpyDeviceToHost)) != hipSuccess)
    return map_err(e);
  if ((e = hipMemset(ws->status, 0, sizeof(uint32_t))) != hipSuccess) return map_err(e);
  *device_status = v;
  return LYAF_OK;
}

}  // extern "C"

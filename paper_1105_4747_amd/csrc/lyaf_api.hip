// lyaf_api.hip -- the C ABI declared in include/lyaf.h: host-side validation,
// per-(device, stream) workspaces, work lists, and the kernel launches.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <sys/stat.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <utility>
#include <vector>

#include "lyaf_internal.h"

namespace lyaf {
namespace {

std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, Workspace *> g_ws;

// A work list uploaded for one workspace and tile length: host mirrors, pinned
// staging and the device copies.  The forward (1024-target tiles by default)
// and the adjoint (512) keep one list each, so calls that alternate between
// them reuse their lists without re-uploading or synchronising.
struct HostPlan {
  int tile = 0;                    // targets per work item
  std::vector<int64_t> offsets;    // [S+1]
  std::vector<int64_t> item_base;  // [S+1]
  int64_t n_items = 0;
  // pinned staging
  int64_t *h_off = nullptr;
  int2 *h_items = nullptr;
  int64_t *h_ib = nullptr;
  int64_t h_off_cap = 0, h_items_cap = 0, h_ib_cap = 0;
  // device copies
  int64_t *d_off = nullptr;
  int2 *d_items = nullptr;
  int64_t *d_ib = nullptr;
  int64_t d_off_cap = 0, d_items_cap = 0, d_ib_cap = 0;
};
std::map<std::pair<Workspace *, int>, HostPlan> g_plans;

int map_err(hipError_t e) {
  if (e == hipSuccess) return LYAF_OK;
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return LYAF_ENOMEM;
  return LYAF_EDEVICE;
}

// Opt-in kernel timing (lyaf_kernel_timing): while enabled, each launch site
// of the entry points records a pair of events around its kernels on the
// caller's stream, under a name; reading a name sums the elapsed times of its
// recorded pairs.  Launches under stream capture are not recorded.
struct TimedLaunch {
  std::string name;
  hipEvent_t start, stop;
};
struct KernelTimer {
  bool on = false;
  std::vector<TimedLaunch> rec;
  std::vector<hipEvent_t> pool;
};
KernelTimer g_kt;
constexpr size_t kMaxTimedLaunches = 1 << 16;

hipEvent_t timer_event() {
  if (!g_kt.pool.empty()) {
    hipEvent_t e = g_kt.pool.back();
    g_kt.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  return hipEventCreate(&e) == hipSuccess ? e : nullptr;
}

template <typename F>
hipError_t timed(const char *name, hipStream_t st, F &&launch) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (!g_kt.on || g_kt.rec.size() >= kMaxTimedLaunches ||
      hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
    return launch();
  hipEvent_t a = timer_event(), b = timer_event();
  if (!a || !b) {
    if (a) g_kt.pool.push_back(a);
    if (b) g_kt.pool.push_back(b);
    return launch();
  }
  hipError_t e = hipEventRecord(a, st);
  if (e != hipSuccess) return e;
  if ((e = launch()) != hipSuccess) return e;
  if ((e = hipEventRecord(b, st)) != hipSuccess) return e;
  g_kt.rec.push_back({name, a, b});
  return hipSuccess;
}

// As timed(), for a launch that takes the events itself and has the runtime
// set them at its kernel's own start and end (hipExtLaunchKernel): no launch
// gap enters the time.  launch(nullptr, nullptr) when not timing.
template <typename F>
hipError_t timed_kernel(const char *name, hipStream_t st, F &&launch) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (!g_kt.on || g_kt.rec.size() >= kMaxTimedLaunches ||
      hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
    return launch(nullptr, nullptr);
  hipEvent_t a = timer_event(), b = timer_event();
  if (!a || !b) {
    if (a) g_kt.pool.push_back(a);
    if (b) g_kt.pool.push_back(b);
    return launch(nullptr, nullptr);
  }
  hipError_t e = launch(a, b);
  if (e != hipSuccess) return e;
  g_kt.rec.push_back({name, a, b});
  return hipSuccess;
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
      (e = hipMalloc((void **)&w->partials, sizeof(double) * kPartialsDoubles)) != hipSuccess ||
      (e = hipMalloc((void **)&w->norm, sizeof(NormState) * (kNormPasses + 2))) != hipSuccess ||
      (e = hipMalloc((void **)&w->ratio, sizeof(double))) != hipSuccess ||
      (e = hipMemset(w->status, 0, sizeof(uint32_t))) != hipSuccess ||
      (e = hipMemset(w->norm, 0, sizeof(NormState) * (kNormPasses + 2))) != hipSuccess ||
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
  if (((prm->flags >> 8) & 0xFu) > (uint32_t)kNumTauVariants) return LYAF_EINVAL;
  if (prm->flags & ~(LYAF_FLAG_PLAIN | LYAF_FLAG_PER_SKEWER | LYAF_FLAG_PERSISTENT | 0xF00u))
    return LYAF_EINVAL;
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
int ensure_plan(Workspace *ws, const lyaf_skewers *sk, int tile, HostPlan **out) {
  HostPlan &hp = g_plans[std::make_pair(ws, tile)];
  *out = &hp;
  const int64_t S = sk->n_skewers;
  if (hp.tile == tile && (int64_t)hp.offsets.size() == S + 1 &&
      memcmp(hp.offsets.data(), sk->offsets, sizeof(int64_t) * (size_t)(S + 1)) == 0)
    return LYAF_OK;
  hipError_t e;
  // the pinned staging buffers may still feed an earlier copy on this stream
  if ((e = hipStreamSynchronize(ws->stream)) != hipSuccess) return map_err(e);
  hp.tile = tile;
  hp.offsets.assign(sk->offsets, sk->offsets + S + 1);
  hp.item_base.assign((size_t)S + 1, 0);
  int64_t ni = 0;
  for (int64_t s = 0; s < S; ++s) {
    hp.item_base[s] = ni;
    ni += (hp.offsets[s + 1] - hp.offsets[s] + tile - 1) / tile;
  }
  hp.item_base[S] = ni;
  hp.n_items = ni;
  if ((e = grow_host(hp.h_off, hp.h_off_cap, S + 1)) != hipSuccess ||
      (e = grow_host(hp.h_ib, hp.h_ib_cap, S + 1)) != hipSuccess ||
      (e = grow_host(hp.h_items, hp.h_items_cap, ni)) != hipSuccess ||
      (e = grow_dev(hp.d_off, hp.d_off_cap, S + 1)) != hipSuccess ||
      (e = grow_dev(hp.d_ib, hp.d_ib_cap, S + 1)) != hipSuccess ||
      (e = grow_dev(hp.d_items, hp.d_items_cap, ni)) != hipSuccess ||
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
  if ((e = hipMemcpyAsync(hp.d_off, hp.h_off, sizeof(int64_t) * (size_t)(S + 1),
                          hipMemcpyHostToDevice, ws->stream)) != hipSuccess ||
      (e = hipMemcpyAsync(hp.d_ib, hp.h_ib, sizeof(int64_t) * (size_t)(S + 1),
                          hipMemcpyHostToDevice, ws->stream)) != hipSuccess ||
      (ni > 0 && (e = hipMemcpyAsync(hp.d_items, hp.h_items, sizeof(int2) * (size_t)ni,
                                     hipMemcpyHostToDevice, ws->stream)) != hipSuccess)) {
    hp.offsets.clear();
    return map_err(e);
  }
  return LYAF_OK;
}

// The instrument work list uploaded for one workspace and direction (forward:
// one item per skewer with bins; backward: one per pixel tile), with its device
// copies.
struct HostInsPlan {
  std::vector<int64_t> offsets, out_offsets;  // [S+1] each
  int64_t n_items = 0;
  int64_t n_sk = 0;   // backward: skewers for the per-skewer kernel (after the items)
  int max_bins = 0;   // the most bins of those skewers
  int64_t *h_off = nullptr, *h_oo = nullptr;
  int2 *h_items = nullptr;
  int64_t h_off_cap = 0, h_oo_cap = 0, h_items_cap = 0;
  int64_t *d_off = nullptr, *d_oo = nullptr;
  int2 *d_items = nullptr;
  int64_t d_off_cap = 0, d_oo_cap = 0, d_items_cap = 0;
};
std::map<std::pair<Workspace *, bool>, HostInsPlan> g_ins_plans;

int check_ins(int64_t S, const int64_t *offsets, const float *dv,
              const lyaf_instrument_params *ip, const int64_t *out_offsets, int64_t *P_out,
              int64_t *Pout_out) {
  if (!ip || S < 0) return LYAF_EINVAL;
  if (!(ip->fwhm_kms >= 0.0) || !isfinite(ip->fwhm_kms)) return LYAF_EINVAL;
  if (!(ip->bin_kms > 0.0) || !isfinite(ip->bin_kms)) return LYAF_EINVAL;
  if (!isfinite(ip->v_start_kms)) return LYAF_EINVAL;
  if (!(ip->noise_sigma >= 0.0) || !isfinite(ip->noise_sigma)) return LYAF_EINVAL;
  if (!(ip->window_k >= 0.0) || !isfinite(ip->window_k)) return LYAF_EINVAL;
  int64_t P = 0, Po = 0;
  if (S > 0) {
    if (!offsets || !out_offsets || !dv) return LYAF_EINVAL;
    if (offsets[0] != 0 || out_offsets[0] != 0) return LYAF_EINVAL;
    for (int64_t s = 0; s < S; ++s) {
      const int64_t n = offsets[s + 1] - offsets[s];
      const int64_t no = out_offsets[s + 1] - out_offsets[s];
      if (n < 0 || n > (int64_t(1) << 24) || no < 0) return LYAF_EINVAL;
      if (no > 0 && n == 0) return LYAF_EINVAL;
    }
    P = offsets[S];
    Po = out_offsets[S];
  }
  *P_out = P;
  *Pout_out = Po;
  return LYAF_OK;
}

// Upload the offsets and the (skewer, item) list of the instrument kernels,
// unless the workspace already holds this exact list.
int ensure_ins_plan(Workspace *ws, int64_t S, const int64_t *offsets, const int64_t *out_offsets,
                    bool backward, HostInsPlan **out) {
  HostInsPlan &hp = g_ins_plans[std::make_pair(ws, backward)];
  *out = &hp;
  if ((int64_t)hp.offsets.size() == S + 1 &&
      memcmp(hp.offsets.data(), offsets, sizeof(int64_t) * (size_t)(S + 1)) == 0 &&
      memcmp(hp.out_offsets.data(), out_offsets, sizeof(int64_t) * (size_t)(S + 1)) == 0)
    return LYAF_OK;
  hipError_t e;
  // the pinned staging buffers may still feed an earlier copy on this stream
  if ((e = hipStreamSynchronize(ws->stream)) != hipSuccess) return map_err(e);
  hp.offsets.clear();
  int64_t ni = 0, nf = 0, max_bins = 0;
  for (int64_t s = 0; s < S; ++s) {
    const int64_t n = offsets[s + 1] - offsets[s], no = out_offsets[s + 1] - out_offsets[s];
    ni += ins_items_per_skewer(n, no, backward);
    if (backward && ins_bwd_skewer_item(n, no)) {
      ++nf;
      max_bins = std::max(max_bins, no);
    }
  }
  if (ni + nf > INT32_MAX) return LYAF_EINVAL;
  if ((e = grow_host(hp.h_off, hp.h_off_cap, S + 1)) != hipSuccess ||
      (e = grow_host(hp.h_oo, hp.h_oo_cap, S + 1)) != hipSuccess ||
      (e = grow_host(hp.h_items, hp.h_items_cap, ni + nf)) != hipSuccess ||
      (e = grow_dev(hp.d_off, hp.d_off_cap, S + 1)) != hipSuccess ||
      (e = grow_dev(hp.d_oo, hp.d_oo_cap, S + 1)) != hipSuccess ||
      (e = grow_dev(hp.d_items, hp.d_items_cap, ni + nf)) != hipSuccess)
    return map_err(e);
  memcpy(hp.h_off, offsets, sizeof(int64_t) * (size_t)(S + 1));
  memcpy(hp.h_oo, out_offsets, sizeof(int64_t) * (size_t)(S + 1));
  int64_t k = 0;
  for (int64_t s = 0; s < S; ++s) {
    const int c = ins_items_per_skewer(offsets[s + 1] - offsets[s],
                                       out_offsets[s + 1] - out_offsets[s], backward);
    for (int t = 0; t < c; ++t) hp.h_items[k++] = make_int2((int)s, t);
  }
  if (backward)
    for (int64_t s = 0; s < S; ++s)
      if (ins_bwd_skewer_item(offsets[s + 1] - offsets[s], out_offsets[s + 1] - out_offsets[s]))
        hp.h_items[k++] = make_int2((int)s, 0);
  if ((e = hipMemcpyAsync(hp.d_off, hp.h_off, sizeof(int64_t) * (size_t)(S + 1),
                          hipMemcpyHostToDevice, ws->stream)) != hipSuccess ||
      (e = hipMemcpyAsync(hp.d_oo, hp.h_oo, sizeof(int64_t) * (size_t)(S + 1),
                          hipMemcpyHostToDevice, ws->stream)) != hipSuccess ||
      (ni + nf > 0 &&
       (e = hipMemcpyAsync(hp.d_items, hp.h_items, sizeof(int2) * (size_t)(ni + nf),
                           hipMemcpyHostToDevice, ws->stream)) != hipSuccess))
    return map_err(e);
  hp.offsets.assign(offsets, offsets + S + 1);
  hp.out_offsets.assign(out_offsets, out_offsets + S + 1);
  hp.n_items = ni;
  hp.n_sk = nf;
  hp.max_bins = (int)max_bins;
  return LYAF_OK;
}

// Host mirror of the power-spectrum offsets uploaded to a workspace.
struct HostPsPlan {
  std::vector<int64_t> offsets;  // [S+1]
  int max_n = 0;
  int64_t *h_off = nullptr, *h_mo = nullptr;
  int64_t h_off_cap = 0, h_mo_cap = 0;
};
std::map<Workspace *, HostPsPlan> g_ps_plans;

int ensure_ps_plan(Workspace *ws, int64_t S, const int64_t *offsets, HostPsPlan **out) {
  HostPsPlan &hp = g_ps_plans[ws];
  *out = &hp;
  if ((int64_t)hp.offsets.size() == S + 1 &&
      memcmp(hp.offsets.data(), offsets, sizeof(int64_t) * (size_t)(S + 1)) == 0)
    return LYAF_OK;
  hipError_t e;
  if ((e = hipStreamSynchronize(ws->stream)) != hipSuccess) return map_err(e);
  hp.offsets.clear();
  if ((e = grow_host(hp.h_off, hp.h_off_cap, S + 1)) != hipSuccess ||
      (e = grow_host(hp.h_mo, hp.h_mo_cap, S + 1)) != hipSuccess ||
      (e = grow_dev(ws->ps_off, ws->ps_off_cap, S + 1)) != hipSuccess ||
      (e = grow_dev(ws->ps_mo, ws->ps_mo_cap, S + 1)) != hipSuccess)
    return map_err(e);
  int max_n = 0;
  hp.h_mo[0] = 0;
  for (int64_t s = 0; s < S; ++s) {
    const int64_t n = offsets[s + 1] - offsets[s];
    hp.h_mo[s + 1] = hp.h_mo[s] + n / 2 + 1;
    max_n = std::max(max_n, (int)n);
  }
  memcpy(hp.h_off, offsets, sizeof(int64_t) * (size_t)(S + 1));
  if ((e = hipMemcpyAsync(ws->ps_off, hp.h_off, sizeof(int64_t) * (size_t)(S + 1),
                          hipMemcpyHostToDevice, ws->stream)) != hipSuccess ||
      (e = hipMemcpyAsync(ws->ps_mo, hp.h_mo, sizeof(int64_t) * (size_t)(S + 1),
                          hipMemcpyHostToDevice, ws->stream)) != hipSuccess)
    return map_err(e);
  hp.max_n = max_n;
  hp.offsets.assign(offsets, offsets + S + 1);
  return LYAF_OK;
}

// The shared FFT twiddle table of a workspace, built on first use.
int ensure_twiddles(Workspace *ws, hipStream_t st) {
  if (ws->ps_twiddle) return LYAF_OK;
  hipError_t e = hipMalloc((void **)&ws->ps_twiddle, sizeof(double2) * (kPsMaxN / 4));
  if (e != hipSuccess) {
    ws->ps_twiddle = nullptr;
    return map_err(e);
  }
  return map_err(launch_twiddles(ws->ps_twiddle, st));
}

// Sight-line plan of the field synthesis: the rows y in use (ascending), the
// sight-lines grouped by row (at most kFieldLinesPerGroup per group), with
// device copies; rebuilt only when the grid side or the columns change.
struct HostFieldPlan {
  int64_t n = 0;
  std::vector<int32_t> sx, sy;
  int n_rows = 0, n_groups = 0;
  int *h_rows = nullptr; int4 *h_groups = nullptr; int2 *h_lines = nullptr;
  int *h_first = nullptr;
  int64_t h_rows_cap = 0, h_groups_cap = 0, h_lines_cap = 0, h_first_cap = 0;
  int *d_rows = nullptr; int4 *d_groups = nullptr; int2 *d_lines = nullptr;
  int *d_first = nullptr;  // [rows + 1]: first line of each row
  int *h_row_of_y = nullptr, *d_row_of_y = nullptr;  // [n]: row of y, -1 if none
  int64_t h_row_of_y_cap = 0, d_row_of_y_cap = 0;
  int64_t d_rows_cap = 0, d_groups_cap = 0, d_lines_cap = 0, d_first_cap = 0;
};
std::map<Workspace *, HostFieldPlan> g_field_plans;

int ensure_field_plan(Workspace *ws, int64_t n, int64_t S, const int32_t *sx, const int32_t *sy,
                      HostFieldPlan **out) {
  HostFieldPlan &hp = g_field_plans[ws];
  *out = &hp;
  if (hp.n == n && (int64_t)hp.sx.size() == S &&
      memcmp(hp.sx.data(), sx, sizeof(int32_t) * (size_t)S) == 0 &&
      memcmp(hp.sy.data(), sy, sizeof(int32_t) * (size_t)S) == 0)
    return LYAF_OK;
  hipError_t e;
  if ((e = hipStreamSynchronize(ws->stream)) != hipSuccess) return map_err(e);
  hp.n = 0;
  // sight-lines ordered by row, then by their index
  std::vector<int32_t> order((size_t)S);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t a, int32_t b) { return sy[a] < sy[b]; });
  std::vector<int> rows, first;
  std::vector<int4> groups;
  for (int64_t i = 0; i < S;) {
    const int y = sy[order[(size_t)i]];
    int64_t j = i;
    while (j < S && sy[order[(size_t)j]] == y) ++j;
    const int ri = (int)rows.size();
    rows.push_back(y);
    first.push_back((int)i);
    for (int64_t g = i; g < j; g += kFieldLinesPerGroup)
      groups.push_back(make_int4(ri, (int)g, (int)std::min<int64_t>(kFieldLinesPerGroup, j - g), 0));
    i = j;
  }
  first.push_back((int)S);
  const int64_t nr = (int64_t)rows.size(), ng = (int64_t)groups.size();
  if ((e = grow_host(hp.h_row_of_y, hp.h_row_of_y_cap, n)) != hipSuccess ||
      (e = grow_dev(hp.d_row_of_y, hp.d_row_of_y_cap, n)) != hipSuccess ||
      (e = grow_host(hp.h_first, hp.h_first_cap, nr + 1)) != hipSuccess ||
      (e = grow_dev(hp.d_first, hp.d_first_cap, nr + 1)) != hipSuccess ||
      (e = grow_host(hp.h_rows, hp.h_rows_cap, nr)) != hipSuccess ||
      (e = grow_host(hp.h_groups, hp.h_groups_cap, ng)) != hipSuccess ||
      (e = grow_host(hp.h_lines, hp.h_lines_cap, S)) != hipSuccess ||
      (e = grow_dev(hp.d_rows, hp.d_rows_cap, nr)) != hipSuccess ||
      (e = grow_dev(hp.d_groups, hp.d_groups_cap, ng)) != hipSuccess ||
      (e = grow_dev(hp.d_lines, hp.d_lines_cap, S)) != hipSuccess)
    return map_err(e);
  std::copy(rows.begin(), rows.end(), hp.h_rows);
  std::copy(first.begin(), first.end(), hp.h_first);
  std::fill(hp.h_row_of_y, hp.h_row_of_y + n, -1);
  for (int64_t r = 0; r < nr; ++r) hp.h_row_of_y[rows[(size_t)r]] = (int)r;
  std::copy(groups.begin(), groups.end(), hp.h_groups);
  for (int64_t i = 0; i < S; ++i)
    hp.h_lines[i] = make_int2(order[(size_t)i], sx[order[(size_t)i]]);
  if ((e = hipMemcpyAsync(hp.d_row_of_y, hp.h_row_of_y, sizeof(int) * (size_t)n,
                          hipMemcpyHostToDevice, ws->stream)) != hipSuccess ||
      (e = hipMemcpyAsync(hp.d_first, hp.h_first, sizeof(int) * (size_t)(nr + 1),
                          hipMemcpyHostToDevice, ws->stream)) != hipSuccess ||
      (nr > 0 && (e = hipMemcpyAsync(hp.d_rows, hp.h_rows, sizeof(int) * (size_t)nr,
                                     hipMemcpyHostToDevice, ws->stream)) != hipSuccess) ||
      (ng > 0 && (e = hipMemcpyAsync(hp.d_groups, hp.h_groups, sizeof(int4) * (size_t)ng,
                                     hipMemcpyHostToDevice, ws->stream)) != hipSuccess) ||
      (S > 0 && (e = hipMemcpyAsync(hp.d_lines, hp.h_lines, sizeof(int2) * (size_t)S,
                                    hipMemcpyHostToDevice, ws->stream)) != hipSuccess))
    return map_err(e);
  hp.n_rows = (int)nr;
  hp.n_groups = (int)ng;
  hp.sx.assign(sx, sx + S);
  hp.sy.assign(sy, sy + S);
  hp.n = n;
  return LYAF_OK;
}

InsArgs make_ins_args(Workspace *ws, const HostInsPlan *hp, const float *dv,
                      const lyaf_instrument_params *ip) {
  InsArgs a;
  a.offsets = hp->d_off;
  a.out_offsets = hp->d_oo;
  a.dv = dv;
  a.in = nullptr;
  a.out = nullptr;
  a.noise = nullptr;
  a.fwhm = ip->fwhm_kms;
  a.bin = ip->bin_kms;
  a.inv_bin = 1.0 / ip->bin_kms;
  a.v_start = ip->v_start_kms;
  a.sigma = ip->noise_sigma;
  a.window_k = ip->window_k;
  a.status = ws->status;
  return a;
}

// offsets_dev: the device copy of the batch's offsets [S+1].
Batch make_batch(const lyaf_skewers *sk, const lyaf_params *prm, Workspace *ws,
                 const int64_t *offsets_dev) {
  Batch b;
  b.delta = sk->delta;
  b.vpec = sk->vpec;
  b.dv = sk->dv;
  b.T0 = sk->T0;
  b.gamma = sk->gamma;
  b.offsets = offsets_dev;
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
  const uint32_t shape = (prm->flags >> 8) & 0xFu;  // validated by check_args
  const int variant = shape ? (int)shape - 1 : kTauVariantDefault;
  HostPlan *hp = nullptr;
  if ((rc = ensure_plan(ws, sk, kTauVariants[variant].tile, &hp))) return rc;
  const Batch b = make_batch(sk, prm, ws, hp->d_off);
  hipError_t e = timed("reach", st, [&] { return launch_reach(b, st); });
  if (e != hipSuccess) return map_err(e);
  const int64_t S = sk->n_skewers;
  if (prm->flags & LYAF_FLAG_PLAIN) {
    for (int64_t s = 0; s < S && e == hipSuccess; ++s)
      e = timed("tau_plain", st, [&] {
        return launch_tau_plain(b, s, hp->offsets[s + 1] - hp->offsets[s], tau_out, st);
      });
  } else if (prm->flags & LYAF_FLAG_PER_SKEWER) {
    for (int64_t s = 0; s < S && e == hipSuccess; ++s)
      e = timed("tau", st, [&] {
        return launch_tau_window(b, hp->d_items + hp->item_base[s],
                                 hp->item_base[s + 1] - hp->item_base[s], tau_out, st, variant);
      });
  } else if (prm->flags & LYAF_FLAG_PERSISTENT) {
    if (!ws->queue && (e = hipMalloc((void **)&ws->queue, sizeof(unsigned int))) != hipSuccess)
      return map_err(e);
    const int pg = tau_persistent_grid(variant);
    if (pg <= 0) return LYAF_EDEVICE;
    e = timed("tau", st, [&] {
      return launch_tau_window(b, hp->d_items, hp->n_items, tau_out, st, variant, pg, ws->queue);
    });
  } else {
    e = timed_kernel("tau", st, [&](hipEvent_t e0, hipEvent_t e1) {
      return launch_tau_window(b, hp->d_items, hp->n_items, tau_out, st, variant, 0, nullptr, e0,
                               e1);
    });
  }
  return map_err(e);
}

int lyaf_normalise_mean_flux(int64_t n_pix, float *tau_inout, float *F_out, double target_F,
                             double *A_dev, void *stream) {
  if (n_pix <= 0 || n_pix > kMaxNormPixels || !tau_inout || !A_dev) return LYAF_EINVAL;
  if (!(target_F > 0.0 && target_F < 1.0)) return LYAF_EINVAL;
  if (F_out == tau_inout) return LYAF_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  hipStream_t st = (hipStream_t)stream;
  Workspace *ws = nullptr;
  int rc = get_ws(st, &ws);
  if (rc) return rc;
  return map_err(timed("normalise", st, [&] {
    return launch_norm(n_pix, tau_inout, F_out, target_F, A_dev, *ws, st);
  }));
}

int lyaf_normalise_mean_flux_noalloc(int64_t n_pix, float *tau_inout, float *F_out,
                                     double target_F, double *A_dev, uint32_t *status_dev,
                                     void *stream) {
  if (n_pix <= 0 || n_pix > kMaxNormPixels || !tau_inout || !A_dev) return LYAF_EINVAL;
  if (!(target_F > 0.0 && target_F < 1.0)) return LYAF_EINVAL;
  if (F_out == tau_inout) return LYAF_EINVAL;
  // no workspace, no lock, no timing events: only kernel launches
  return map_err(launch_norm_noalloc(n_pix, tau_inout, F_out, target_F, A_dev, status_dev,
                                     (hipStream_t)stream));
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
  return map_err(timed("normalise_backward", st, [&] {
    return launch_norm_backward(n_pix, tau_raw, A_dev, grad_F, grad_tau_scaled,
                                implicit_A ? 1 : 0, grad_tau_raw_out, *ws, st);
  }));
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
  if ((rc = ensure_plan(ws, sk, kTauTile, &hp))) return rc;
  hipError_t e = grow_dev(ws->gpart, ws->gpart_cap, 2 * std::max<int64_t>(hp->n_items, 1));
  if (e != hipSuccess) return map_err(e);
  const Batch b = make_batch(sk, prm, ws, hp->d_off);
  if ((e = timed("reach", st, [&] { return launch_reach(b, st); })) != hipSuccess)
    return map_err(e);
  if (hp->n_items == 0) {
    // every skewer is empty: the per-skewer sums are zero
    if (grad_T0 && (e = hipMemsetAsync(grad_T0, 0, sizeof(double) * (size_t)sk->n_skewers, st)))
      return map_err(e);
    if (grad_gamma &&
        (e = hipMemsetAsync(grad_gamma, 0, sizeof(double) * (size_t)sk->n_skewers, st)))
      return map_err(e);
    return LYAF_OK;
  }
  return map_err(timed("tau_adjoint", st, [&] {
    return launch_tau_adjoint(b, hp->d_items, hp->n_items, hp->d_ib, grad_tau_raw, grad_delta,
                              grad_vpec, grad_T0, grad_gamma, ws->gpart, st);
  }));
}

int lyaf_instrument(int64_t n_skewers, const int64_t *offsets, const float *dv, const float *F,
                    const lyaf_instrument_params *ip, const int64_t *out_offsets,
                    const float *noise, float *F_obs, void *stream) {
  int64_t P = 0, Po = 0;
  int rc = check_ins(n_skewers, offsets, dv, ip, out_offsets, &P, &Po);
  if (rc) return rc;
  if (Po == 0) return LYAF_OK;
  if (!F || !F_obs || (ip->noise_sigma > 0.0 && !noise)) return LYAF_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  hipStream_t st = (hipStream_t)stream;
  Workspace *ws = nullptr;
  if ((rc = get_ws(st, &ws))) return rc;
  HostInsPlan *hp = nullptr;
  if ((rc = ensure_ins_plan(ws, n_skewers, offsets, out_offsets, false, &hp))) return rc;
  InsArgs a = make_ins_args(ws, hp, dv, ip);
  a.in = F;
  a.out = F_obs;
  a.noise = ip->noise_sigma > 0.0 ? noise : nullptr;
  return map_err(timed("instrument", st, [&] {
    return launch_instrument(a, hp->d_items, hp->n_items, nullptr, 0, 0, false, st);
  }));
}

int lyaf_instrument_backward(int64_t n_skewers, const int64_t *offsets, const float *dv,
                             const lyaf_instrument_params *ip, const int64_t *out_offsets,
                             const float *grad_obs, float *grad_F, void *stream) {
  int64_t P = 0, Po = 0;
  int rc = check_ins(n_skewers, offsets, dv, ip, out_offsets, &P, &Po);
  if (rc) return rc;
  if (P == 0) return LYAF_OK;
  if (!grad_F || (Po > 0 && !grad_obs)) return LYAF_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  hipStream_t st = (hipStream_t)stream;
  Workspace *ws = nullptr;
  if ((rc = get_ws(st, &ws))) return rc;
  HostInsPlan *hp = nullptr;
  if ((rc = ensure_ins_plan(ws, n_skewers, offsets, out_offsets, true, &hp))) return rc;
  InsArgs a = make_ins_args(ws, hp, dv, ip);
  a.in = grad_obs;
  a.out = grad_F;
  return map_err(timed("instrument_backward", st, [&] {
    return launch_instrument(a, hp->d_items, hp->n_items, hp->d_items + hp->n_items, hp->n_sk,
                             hp->max_bins, true, st);
  }));
}

int lyaf_flux_pdf(int64_t n_pix, const float *F, int64_t *counts, void *stream) {
  if (n_pix < 0 || !counts || (n_pix > 0 && !F)) return LYAF_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  hipStream_t st = (hipStream_t)stream;
  Workspace *ws = nullptr;
  int rc = get_ws(st, &ws);
  if (rc) return rc;
  hipError_t e = grow_dev(ws->pdf_part, ws->pdf_part_cap, (int64_t)kPdfMaxBlocks * kPdfCountSlots);
  if (e != hipSuccess) return map_err(e);
  return map_err(
      timed("flux_pdf", st, [&] { return launch_flux_pdf(n_pix, F, ws->pdf_part, counts, st); }));
}

int lyaf_flux_power(int64_t n_skewers, const int64_t *offsets, const float *dv, const float *F,
                    double mean_F, float *power, void *stream) {
  if (n_skewers < 0 || !(mean_F > 0.0) || !isfinite(mean_F)) return LYAF_EINVAL;
  if (n_skewers == 0) return LYAF_OK;
  if (!offsets || !dv || !F || !power || offsets[0] != 0) return LYAF_EINVAL;
  for (int64_t s = 0; s < n_skewers; ++s) {
    const int64_t n = offsets[s + 1] - offsets[s];
    if (n < 2 || n > kPsMaxN || (n & (n - 1)) != 0) return LYAF_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  hipStream_t st = (hipStream_t)stream;
  Workspace *ws = nullptr;
  int rc = get_ws(st, &ws);
  if (rc) return rc;
  HostPsPlan *hp = nullptr;
  if ((rc = ensure_ps_plan(ws, n_skewers, offsets, &hp))) return rc;
  if ((rc = ensure_twiddles(ws, st))) return rc;
  return map_err(timed("flux_power", st, [&] {
    return launch_flux_power(n_skewers, hp->max_n, F, ws->ps_off, ws->ps_mo, dv,
                             1.0 / mean_F, ws->ps_twiddle, power, ws->status, st);
  }));
}

int lyaf_field_skewers(const lyaf_field_params *fp, const void *modes, const double *pk,
                       int64_t n_lines, const int32_t *sx, const int32_t *sy, float *delta_b,
                       float *v_z, void *stream) {
  if (!fp || n_lines < 0) return LYAF_EINVAL;
  const int64_t N = fp->n;
  if (N < 4 || N > kFieldMaxN || (N & (N - 1)) != 0) return LYAF_EINVAL;
  if (!(fp->box > 0.0) || !isfinite(fp->box) || !isfinite(fp->amp)) return LYAF_EINVAL;
  if (!(fp->k_F > 0.0) || !isfinite(fp->E_plus)) return LYAF_EINVAL;  // k_F = +INF allowed
  if (!(fp->dk > 0.0) || !isfinite(fp->dk)) return LYAF_EINVAL;
  if (fp->n_table < 1 || fp->n_table > INT32_MAX) return LYAF_EINVAL;
  if (n_lines == 0) return LYAF_OK;
  if (n_lines > INT32_MAX || !modes || !pk || !sx || !sy || !delta_b || !v_z)
    return LYAF_EINVAL;
  for (int64_t s = 0; s < n_lines; ++s)
    if (sx[s] < 0 || sx[s] >= N || sy[s] < 0 || sy[s] >= N) return LYAF_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  hipStream_t st = (hipStream_t)stream;
  Workspace *ws = nullptr;
  int rc = get_ws(st, &ws);
  if (rc) return rc;
  HostFieldPlan *hp = nullptr;
  if ((rc = ensure_field_plan(ws, N, n_lines, sx, sy, &hp))) return rc;
  if ((rc = ensure_twiddles(ws, st))) return rc;
  const int64_t H = N / 2 + 1;
  hipError_t e;
  int ky_resident = 0;
  if ((e = field_kernel_attributes(&ky_resident)) != hipSuccess ||
      (e = grow_dev(ws->field_T, ws->field_T_cap, 2 * (int64_t)hp->n_rows * N * H)) !=
          hipSuccess ||
      (e = grow_dev(ws->field_C, ws->field_C_cap, 2 * n_lines * H)) != hipSuccess)
    return map_err(e);
  FieldArgs a;
  a.modes = static_cast<const float2 *>(modes);
  a.pk = pk;
  a.N = (int)N;
  a.H = (int)H;
  a.n_table = (int)fp->n_table;
  a.n_rows = hp->n_rows;
  const double kfun = 2.0 * M_PI / fp->box;
  a.kfun = (float)kfun;
  a.inv_dk = (float)(1.0 / fp->dk);
  a.amp = (float)fp->amp;
  a.kfun2_inv_kF2 = isinf(fp->k_F) ? 0.f : (float)(kfun * kfun / (fp->k_F * fp->k_F));
  a.E_over_kfun = (float)(fp->E_plus / kfun);
  a.inv_n3 = 1.0 / ((double)N * (double)N * (double)N);
  a.rows = hp->d_rows;
  a.groups = hp->d_groups;
  a.lines = hp->d_lines;
  a.Tb = ws->field_T;
  a.Tv = ws->field_T + (int64_t)hp->n_rows * N * H;
  a.Cb = ws->field_C;
  a.Cv = ws->field_C + n_lines * H;
  a.delta_b = delta_b;
  a.v_z = v_z;
  a.twiddle = ws->ps_twiddle;
  if ((e = timed("field_ky", st, [&] { return launch_field_ky(a, ky_resident, st); })) !=
          hipSuccess ||
      (e = timed("field_kx", st, [&] { return launch_field_kx(a, hp->n_groups, st); })) !=
          hipSuccess)
    return map_err(e);
  return map_err(timed("field_z", st, [&] { return launch_field_z(a, (int)n_lines, st); }));
}

int lyaf_flux_power_3d(const lyaf_power3d_params *pp, int64_t n_lines, const float *F,
                       const int32_t *sx, const int32_t *sy, const double *weights,
                       double *counts, double *k_mean, double *p_true, double *p_box,
                       void *stream) {
  if (!pp) return LYAF_EINVAL;
  const int64_t n = pp->n;
  if (n < 4 || n > kP3dMaxN || (n & (n - 1)) != 0) return LYAF_EINVAL;
  if (!(pp->box > 0.0) || !isfinite(pp->box)) return LYAF_EINVAL;
  if (!(pp->mean_F > 0.0) || !isfinite(pp->mean_F)) return LYAF_EINVAL;
  if (!(pp->p_noise >= 0.0) || !isfinite(pp->p_noise)) return LYAF_EINVAL;
  if (pp->n_bins < 1 || pp->n_bins > INT32_MAX) return LYAF_EINVAL;
  if (n_lines < 1 || n_lines > INT32_MAX || !F || !sx || !sy) return LYAF_EINVAL;
  if (!counts || !k_mean || !p_true || !p_box) return LYAF_EINVAL;
  for (int64_t s = 0; s < n_lines; ++s)
    if (sx[s] < 0 || sx[s] >= n || sy[s] < 0 || sy[s] >= n) return LYAF_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  hipStream_t st = (hipStream_t)stream;
  Workspace *ws = nullptr;
  int rc = get_ws(st, &ws);
  if (rc) return rc;
  HostFieldPlan *hp = nullptr;
  if ((rc = ensure_field_plan(ws, n, n_lines, sx, sy, &hp))) return rc;
  if ((rc = ensure_twiddles(ws, st))) return rc;
  const int64_t H = n / 2 + 1;
  const int nb = p3d_shell_bins((int)n, (int)pp->n_bins);
  int y_grid = 0;
  hipError_t e;
  if ((e = p3d_kernel_attributes((int)n, nb, &y_grid)) != hipSuccess) return map_err(e);
  const int C = p3d_y_columns((int)n);
  y_grid = (int)std::min<int64_t>(y_grid, n * ((H + C - 1) / C));
  const int64_t n_c = n_lines * H + n * (int64_t)hp->n_rows * H;  // G, D1
  const int64_t p1d_parts = (n_lines + kP3dP1dChunk - 1) / kP3dP1dChunk;
  // P1d, P2d, data shells, geometry shells, P1d partials
  const int64_t n_r = H + n * n + 2 * ((int64_t)y_grid * 2 * nb) + p1d_parts * H;
  const bool need_geom = ws->p3d_geom_n != (int)n || ws->p3d_geom_nb != nb;
  if (need_geom) ws->p3d_geom_n = ws->p3d_geom_nb = 0;
  if ((e = grow_dev(ws->p3d_c, ws->p3d_c_cap, n_c)) != hipSuccess ||
      (e = grow_dev(ws->p3d_r, ws->p3d_r_cap, n_r)) != hipSuccess ||
      (e = grow_dev(ws->p3d_geom, ws->p3d_geom_cap, 2 * (int64_t)nb)) != hipSuccess)
    return map_err(e);
  P3dArgs a;
  a.F = F;
  a.w = weights;
  a.n = (int)n;
  a.H = (int)H;
  a.n_rows = hp->n_rows;
  a.n_lines = (int)n_lines;
  a.n_bins = (int)pp->n_bins;
  a.inv_mean = 1.0 / pp->mean_F;
  a.L = pp->box;
  a.p_noise = pp->p_noise;
  a.rows = hp->d_rows;
  a.row_first = hp->d_first;
  a.lines = hp->d_lines;
  a.G = ws->p3d_c;
  a.D1 = ws->p3d_c + n_lines * H;
  a.P1d = ws->p3d_r;
  a.P2d = ws->p3d_r + H;
  a.shells = ws->p3d_r + H + n * n;
  a.geom_part = a.shells + (int64_t)y_grid * 2 * nb;
  a.p1d_part = a.geom_part + (int64_t)y_grid * 2 * nb;
  a.geom = ws->p3d_geom;
  a.row_of_y = hp->d_row_of_y;
  a.counts = counts;
  a.k_mean = k_mean;
  a.p_true = p_true;
  a.p_box = p_box;
  a.twiddle = ws->ps_twiddle;
  if ((e = timed("flux_power_3d", st,
                 [&] { return launch_power3d(a, y_grid, need_geom, st); })) != hipSuccess)
    return map_err(e);
  ws->p3d_geom_n = (int)n;
  ws->p3d_geom_nb = nb;
  return LYAF_OK;
}

double lyaf_angstrom_to_kms(double dlambda_angstrom, double z) {
  return kSpeedOfLightKms * dlambda_angstrom / (kLymanAlphaAngstrom * (1.0 + z));
}

double lyaf_lya_lyb_path_kms(double proximity_kms) {
  return kSpeedOfLightKms * log(kLymanAlphaAngstrom / kLymanBetaAngstrom) - proximity_kms;
}

int lyaf_kernel_timing(int enable) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto &r : g_kt.rec) {
    g_kt.pool.push_back(r.start);
    g_kt.pool.push_back(r.stop);
  }
  g_kt.rec.clear();
  g_kt.on = enable != 0;
  return LYAF_OK;
}

int lyaf_kernel_timing_read(const char *name, double *total_ms, int64_t *count) {
  if (!name || !total_ms || !count) return LYAF_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  double sum = 0.0;
  int64_t n = 0;
  std::vector<TimedLaunch> keep;
  for (auto &r : g_kt.rec) {
    if (r.name != name) {
      keep.push_back(r);
      continue;
    }
    float ms = 0.f;
    hipError_t e = hipEventSynchronize(r.stop);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.start, r.stop);
    if (e != hipSuccess) return map_err(e);
    sum += (double)ms;
    ++n;
    g_kt.pool.push_back(r.start);
    g_kt.pool.push_back(r.stop);
  }
  g_kt.rec.swap(keep);
  *total_ms = sum;
  *count = n;
  return LYAF_OK;
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

// ===========================================================================
// Plans.
namespace lyaf {
namespace {

struct Candidate {
  int variant;
  int persistent;  // 1: persistent work-queue launch
  double us;
};

std::string tune_cache_path() {
  const char *p = getenv("LYAF_TUNE_CACHE");
  if (p && *p) return p;
  const char *h = getenv("HOME");
  std::string dir = std::string(h && *h ? h : "/tmp") + "/.cache";
  return dir + "/lyaf_tune.txt";
}

bool tune_cache_lookup(const std::string &key, Candidate *c) {
  FILE *f = fopen(tune_cache_path().c_str(), "r");
  if (!f) return false;
  char k[512];
  int v = 0, ps = 0;
  double us = 0;
  bool found = false;
  while (fscanf(f, "%511s %d %d %lf", k, &v, &ps, &us) == 4) {
    if (key == k && v >= 0 && v < kNumTauVariants && (ps == 0 || ps == 1)) {
      c->variant = v;
      c->persistent = ps;
      c->us = us;
      found = true;  // the last matching line wins
    }
  }
  fclose(f);
  return found;
}

void tune_cache_store(const std::string &key, const Candidate &c) {
  const std::string path = tune_cache_path();
  const size_t slash = path.find_last_of('/');
  if (slash != std::string::npos && slash > 0)
    mkdir(path.substr(0, slash).c_str(), 0755);  // best effort, one level
  FILE *f = fopen(path.c_str(), "a");
  if (!f) return;  // an unwritable cache only costs a re-tune later
  fprintf(f, "%s %d %d %.3f\n", key.c_str(), c.variant, c.persistent, c.us);
  fclose(f);
}

}  // namespace
}  // namespace lyaf

struct lyaf_plan {
  int device = -1;
  lyaf_skewers sk{};
  std::vector<int64_t> offsets;
  lyaf_params prm{};
  double target_F = 0.0;
  float *tau_out = nullptr, *F_out = nullptr;
  double *A_dev = nullptr;
  uint32_t flags = 0;
  int64_t P = 0;
  lyaf::Workspace ws;
  int2 *items = nullptr;
  int64_t n_items = 0, items_cap = 0;
  unsigned int *queue = nullptr;
  int variant = lyaf::kTauVariantDefault;
  int persistent_grid = 0;
  bool tuned = false, from_cache = false;
  std::string tune_key;
  std::vector<lyaf::Candidate> timings;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<lyaf::SkewerConst> skc_host;
};

namespace lyaf {
namespace {

void plan_free(lyaf_plan *p) {
  if (!p) return;
  // teardown: errors here leave nothing further to release
  (void)hipDeviceSynchronize();
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  void *bufs[] = {p->items, p->queue, p->ws.status, p->ws.partials, p->ws.norm,
                  p->ws.ratio, p->ws.skc, p->ws.offsets};
  for (void *q : bufs)
    if (q) (void)hipFree(q);
  delete p;
}

// (skewer, tile) work items for a tile length, largest estimated cost first.
// A windowed tile of t targets stages t + 2R sources and evaluates about
// t (t_sub + 2R) pairs; a full-sum tile evaluates t n.
std::vector<int2> build_items(const lyaf_plan *p, int tile) {
  const int64_t S = p->sk.n_skewers;
  std::vector<int2> items;
  std::vector<double> cost;
  for (int64_t s = 0; s < S; ++s) {
    const int64_t n = p->offsets[s + 1] - p->offsets[s];
    const int R = p->skc_host.empty() ? 0 : p->skc_host[s].reach;
    const int64_t nt = (n + tile - 1) / tile;
    for (int64_t t = 0; t < nt; ++t) {
      const double tg = (double)std::min<int64_t>(tile, n - t * tile);
      const bool full = (int64_t)(32 + 2 * R + 24) > n;
      items.push_back(make_int2((int)s, (int)t));
      cost.push_back(full ? tg * (double)n : tg * (double)std::min<int64_t>(n, 64 + 2 * R));
    }
  }
  std::vector<size_t> ord(items.size());
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(),
                   [&](size_t a, size_t b) { return cost[a] > cost[b]; });
  std::vector<int2> out(items.size());
  for (size_t k = 0; k < ord.size(); ++k) out[k] = items[ord[k]];
  return out;
}

hipError_t upload_items(lyaf_plan *p, const std::vector<int2> &items) {
  hipError_t e = grow_dev(p->items, p->items_cap, (int64_t)std::max<size_t>(items.size(), 1));
  if (e != hipSuccess) return e;
  p->n_items = (int64_t)items.size();
  if (items.empty()) return hipSuccess;
  return hipMemcpy(p->items, items.data(), sizeof(int2) * items.size(), hipMemcpyHostToDevice);
}

Batch plan_batch(lyaf_plan *p) { return make_batch(&p->sk, &p->prm, &p->ws, p->ws.offsets); }

hipError_t enqueue_tau(lyaf_plan *p, hipStream_t st) {
  const Batch b = plan_batch(p);
  hipError_t e = launch_reach(b, st);
  if (e != hipSuccess) return e;
  return launch_tau_window(b, p->items, p->n_items, p->tau_out, st, p->variant,
                           p->persistent_grid, p->queue);
}

hipError_t enqueue_forward(lyaf_plan *p, hipStream_t st) {
  hipError_t e = enqueue_tau(p, st);
  if (e != hipSuccess) return e;
  return launch_norm(p->P, p->tau_out, p->F_out, p->target_F, p->A_dev, p->ws, st);
}

std::string make_tune_key(const lyaf_plan *p) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, p->device) != hipSuccess) return "v3|unknown";
  const int64_t S = p->sk.n_skewers;
  const double meanN = S > 0 ? (double)p->P / (double)S : 0.0;
  int maxR = 0;
  for (const auto &k : p->skc_host) maxR = std::max(maxR, k.reach);
  char buf[512];
  snprintf(buf, sizeof(buf), "v3|%s|cu%d|S2^%d|N2^%d|R2^%d|k%g", prop.gcnArchName,
           prop.multiProcessorCount, (int)lround(log2((double)std::max<int64_t>(S, 1))),
           (int)lround(log2(std::max(meanN, 1.0))), (int)lround(log2(std::max(maxR, 1))),
           p->prm.window_k);
  std::string k(buf);
  for (auto &c : k)
    if (c == ' ' || c == ':') c = '_';
  return k;
}

// Time the tau stage of every candidate on the plan's data: after one warm-up,
// kTuneReps replays each between its own pair of events, and the candidate's
// time is their median.  The persistent launch is kept only when it beats the
// best one-workgroup-per-item launch by more than kTuneMargin (its queue costs
// atomics and a reset launch; within the noise the plain grid wins).
constexpr int kTuneReps = 11;
constexpr double kTuneMargin = 0.02;

int autotune(lyaf_plan *p, hipStream_t st) {
  hipEvent_t ev[kTuneReps + 1] = {};
  auto destroy = [&]() {
    for (auto &x : ev)
      if (x) (void)hipEventDestroy(x);
  };
  for (auto &x : ev)
    if (hipEventCreate(&x) != hipSuccess) {
      destroy();
      return LYAF_EDEVICE;
    }
  Candidate best_grid{-1, 0, 1e300}, best_pers{-1, 1, 1e300};
  int rc = LYAF_OK;
  for (int v = 0; v < kNumTauVariants && rc == LYAF_OK; ++v) {
    if (upload_items(p, build_items(p, kTauVariants[v].tile)) != hipSuccess) {
      rc = LYAF_ENOMEM;
      break;
    }
    const int pg = tau_persistent_grid(v);
    for (int ps = 0; ps < 2 && rc == LYAF_OK; ++ps) {
      if (ps && pg <= 0) continue;
      p->variant = v;
      p->persistent_grid = ps ? pg : 0;
      bool ok = enqueue_tau(p, st) == hipSuccess && hipEventRecord(ev[0], st) == hipSuccess;
      for (int r = 0; r < kTuneReps && ok; ++r)
        ok = enqueue_tau(p, st) == hipSuccess && hipEventRecord(ev[r + 1], st) == hipSuccess;
      ok = ok && hipEventSynchronize(ev[kTuneReps]) == hipSuccess;
      double t[kTuneReps];
      for (int r = 0; r < kTuneReps && ok; ++r) {
        float ms = 0.f;
        ok = hipEventElapsedTime(&ms, ev[r], ev[r + 1]) == hipSuccess;
        t[r] = 1e3 * (double)ms;
      }
      if (!ok) {
        rc = LYAF_EDEVICE;
        break;
      }
      std::sort(t, t + kTuneReps);
      const Candidate c{v, ps, t[kTuneReps / 2]};
      p->timings.push_back(c);
      Candidate &best = ps ? best_pers : best_grid;
      if (c.us < best.us) best = c;
    }
  }
  destroy();
  if (rc != LYAF_OK) return rc;
  Candidate best = best_grid;
  if (best_pers.variant >= 0 &&
      (best.variant < 0 || best_pers.us < (1.0 - kTuneMargin) * best.us))
    best = best_pers;
  if (best.variant < 0) return LYAF_EDEVICE;
  p->variant = best.variant;
  p->persistent_grid = best.persistent ? tau_persistent_grid(best.variant) : 0;
  tune_cache_store(p->tune_key, best);
  return LYAF_OK;
}

}  // namespace
}  // namespace lyaf

extern "C" {

int lyaf_plan_create(const lyaf_skewers *sk, const lyaf_params *prm, double target_F,
                     float *tau_out, float *F_out, double *A_dev, uint32_t plan_flags,
                     void *stream, lyaf_plan **plan_out) {
  int64_t P = 0;
  int rc = check_args(sk, prm, &P);
  if (rc) return rc;
  if (!plan_out || P <= 0 || !tau_out || !F_out || !A_dev) return LYAF_EINVAL;
  if (!(target_F > 0.0 && target_F < 1.0) || F_out == tau_out) return LYAF_EINVAL;
  if (plan_flags & ~(LYAF_PLAN_AUTOTUNE | LYAF_PLAN_NO_GRAPH)) return LYAF_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  hipStream_t st = (hipStream_t)stream;
  lyaf_plan *p = new lyaf_plan();
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) {
    delete p;
    return map_err(e);
  }
  const int64_t S = sk->n_skewers;
  p->sk = *sk;
  p->offsets.assign(sk->offsets, sk->offsets + S + 1);
  p->sk.offsets = p->offsets.data();
  p->prm = *prm;
  p->target_F = target_F;
  p->tau_out = tau_out;
  p->F_out = F_out;
  p->A_dev = A_dev;
  p->flags = plan_flags;
  p->P = P;
  if ((e = grow_dev(p->ws.offsets, p->ws.off_cap, S + 1)) != hipSuccess ||
      (e = grow_dev(p->ws.skc, p->ws.skc_cap, S)) != hipSuccess ||
      (e = hipMalloc((void **)&p->ws.status, sizeof(uint32_t))) != hipSuccess ||
      (e = hipMalloc((void **)&p->ws.partials, sizeof(double) * kPartialsDoubles)) != hipSuccess ||
      (e = hipMalloc((void **)&p->ws.norm, sizeof(NormState) * (kNormPasses + 2))) != hipSuccess ||
      (e = hipMalloc((void **)&p->ws.ratio, sizeof(double))) != hipSuccess ||
      (e = hipMalloc((void **)&p->queue, sizeof(unsigned int))) != hipSuccess ||
      (e = hipMemset(p->ws.status, 0, sizeof(uint32_t))) != hipSuccess ||
      (e = hipMemset(p->ws.norm, 0, sizeof(NormState) * (kNormPasses + 2))) != hipSuccess ||
      (e = hipMemset(p->queue, 0, sizeof(unsigned int))) != hipSuccess ||
      (e = hipMemcpy(p->ws.offsets, p->offsets.data(), sizeof(int64_t) * (S + 1),
                     hipMemcpyHostToDevice)) != hipSuccess) {
    plan_free(p);
    return map_err(e);
  }
  // per-skewer reach of the data at hand: it orders the work list by cost
  p->skc_host.resize((size_t)S);
  if ((e = launch_reach(plan_batch(p), st)) != hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess ||
      (S > 0 && (e = hipMemcpy(p->skc_host.data(), p->ws.skc, sizeof(SkewerConst) * S,
                               hipMemcpyDeviceToHost)) != hipSuccess)) {
    plan_free(p);
    return map_err(e);
  }
  p->tune_key = make_tune_key(p);
  Candidate cached{};
  if (plan_flags & LYAF_PLAN_AUTOTUNE) {
    p->tuned = true;
    if (tune_cache_lookup(p->tune_key, &cached)) {
      p->from_cache = true;
      p->variant = cached.variant;
      p->persistent_grid = cached.persistent ? tau_persistent_grid(cached.variant) : 0;
      p->timings.push_back(cached);
    } else if ((rc = autotune(p, st))) {
      plan_free(p);
      return rc;
    }
  } else {
    p->variant = kTauVariantDefault;
    p->persistent_grid = tau_persistent_grid(p->variant);
  }
  if ((e = upload_items(p, build_items(p, kTauVariants[p->variant].tile))) != hipSuccess) {
    plan_free(p);
    return map_err(e);
  }
  if (!(plan_flags & LYAF_PLAN_NO_GRAPH)) {
    hipStream_t cap_st = nullptr;
    if ((e = hipStreamCreateWithFlags(&cap_st, hipStreamNonBlocking)) != hipSuccess) {
      plan_free(p);
      return map_err(e);
    }
    e = hipStreamBeginCapture(cap_st, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      hipError_t el = enqueue_forward(p, cap_st);
      e = hipStreamEndCapture(cap_st, &p->graph);
      if (el != hipSuccess) e = el;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cap_st);
    if (e != hipSuccess) {
      plan_free(p);
      return map_err(e);
    }
  }
  // one execution: the outputs are valid on return
  e = p->exec ? hipGraphLaunch(p->exec, st) : enqueue_forward(p, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    plan_free(p);
    return map_err(e);
  }
  *plan_out = p;
  return LYAF_OK;
}

int lyaf_plan_execute(lyaf_plan *plan, void *stream) {
  if (!plan) return LYAF_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = plan->exec ? hipGraphLaunch(plan->exec, st) : enqueue_forward(plan, st);
  return map_err(e);
}

int lyaf_plan_status(lyaf_plan *plan, void *stream, uint32_t *device_status) {
  if (!plan || !device_status) return LYAF_EINVAL;
  uint32_t v = 0;
  hipError_t e;
  if ((e = hipStreamSynchronize((hipStream_t)stream)) != hipSuccess ||
      (e = hipMemcpy(&v, plan->ws.status, sizeof(uint32_t), hipMemcpyDeviceToHost)) != hipSuccess ||
      (e = hipMemset(plan->ws.status, 0, sizeof(uint32_t))) != hipSuccess)
    return map_err(e);
  *device_status = v;
  return LYAF_OK;
}

int lyaf_plan_describe(const lyaf_plan *plan, char *buf, int64_t buf_len) {
  if (!plan || (buf_len > 0 && !buf) || buf_len < 0) return LYAF_EINVAL;
  const TauVariant &v = kTauVariants[plan->variant];
  std::string t = "[";
  for (size_t k = 0; k < plan->timings.size(); ++k) {
    char c[128];
    snprintf(c, sizeof(c), "%s{\"variant\":%d,\"persistent\":%d,\"us\":%.3f}", k ? "," : "",
             plan->timings[k].variant, plan->timings[k].persistent, plan->timings[k].us);
    t += c;
  }
  t += "]";
  char head[768];
  snprintf(head, sizeof(head),
           "{\"shape\":%d,\"streams\":%d,\"targets_per_lane\":%d,\"tile\":%d,"
           "\"persistent_grid\":%d,"
           "\"items\":%lld,\"graph\":%s,\"tuned\":%s,\"from_cache\":%s,\"key\":\"%s\","
           "\"timings_us\":",
           plan->variant, v.S, v.M, v.tile, plan->persistent_grid, (long long)plan->n_items,
           plan->exec ? "true" : "false", plan->tuned ? "true" : "false",
           plan->from_cache ? "true" : "false", plan->tune_key.c_str());
  std::string out = std::string(head) + t + "}";
  if (buf_len > 0) {
    const size_t n = std::min<size_t>(out.size(), (size_t)buf_len - 1);
    memcpy(buf, out.data(), n);
    buf[n] = 0;
  }
  return (int)out.size();
}

int lyaf_plan_destroy(lyaf_plan *plan) {
  if (!plan) return LYAF_OK;
  std::lock_guard<std::mutex> lk(g_mu);
  plan_free(plan);
  return LYAF_OK;
}

}  // extern "C"

// sale_api.cpp -- host side of the libsale C ABI declared in include/sale.h:
// argument validation, workspace layout, enqueueing of the step kernels on
// the caller's stream, status polling and field export, for both precisions.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>

#include "../../include/sale.h"
#include "sale_impl.h"
#include "sale_pool.h"

using sale::Ctl;
using sale::Mesh;
using sale::Work;

struct sale_ctx {
  sale_config cfg;
  Mesh m;
  hipStream_t stream;
  void *ws;
  size_t ws_bytes;
  Ctl *ctl;
  int precision;
  Work<double> w64;
  Work<float> w32;
  int cur;  // which of the two state buffers holds the current state
  double t_end;
  sale::Launch L;  // launch shape of the step kernels
  // step graphs: kGraphSteps steps captured once per starting buffer parity
  // on a private capture stream, replayed on `stream` by sale_run
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  long long enqueued = 0;  // steps enqueued through sale_run
  // a context of sale_init_static: intermediates in the library's device
  // array, host storage in a static table, no step graphs (every call on it
  // allocates nothing)
  bool is_static = false;
  ~sale_ctx() {
    for (int k = 0; k < 2; k++)
      if (graph[k]) (void)hipGraphExecDestroy(graph[k]);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
  }
};

// Steps per captured graph (even, so that a replay leaves the current state
// in the buffer it started from), and the steps a context runs eagerly before
// it captures one (a short run would not earn the capture back).
constexpr int kGraphSteps = 8;
#ifndef SALE_GRAPH_AFTER
#define SALE_GRAPH_AFTER 128
#endif
constexpr long long kGraphAfter = SALE_GRAPH_AFTER;

namespace sale_host {

thread_local char g_hip_msg[256] = "no HIP error recorded";

int hip_fail(hipError_t e, const char *what) {
  snprintf(g_hip_msg, sizeof(g_hip_msg), "%s: %s", what, hipGetErrorString(e));
  return SALE_EHIP;
}

bool finite_pos(double x) { return isfinite(x) && x > 0.0; }

int validate_config(const sale_config *c) {
  if (!c) return SALE_EINVAL;
  const int32_t lim = 1 << 16;
  if (c->nx < 1 || c->ny < 1 || c->nz < 1 || c->nx > lim || c->ny > lim || c->nz > lim)
    return SALE_EINVAL;
  for (int a = 0; a < 3; a++)
    if (!isfinite(c->lo[a]) || !isfinite(c->hi[a]) || !(c->hi[a] > c->lo[a])) return SALE_EINVAL;
  if (!isfinite(c->gamma) || !(c->gamma > 1.0)) return SALE_EINVAL;
  if (!isfinite(c->cfl) || !(c->cfl > 0.0) || !(c->cfl < 1.0)) return SALE_EINVAL;
  if (!isfinite(c->c_quad) || !(c->c_quad >= 0.0) || !isfinite(c->c_lin) || !(c->c_lin >= 0.0))
    return SALE_EINVAL;
  if (!isfinite(c->t_end) || !(c->t_end >= 0.0)) return SALE_EINVAL;
  if (c->precision != SALE_FP64 && c->precision != SALE_MIXED32) return SALE_EINVAL;
  for (int a = 0; a < 6; a++)
    if (c->bc[a] != SALE_BC_REFLECT) return SALE_EINVAL;
  if (c->remap_order < 0 || c->remap_order > 2) return SALE_EINVAL;
  if (c->mode != SALE_EULERIAN && c->mode != SALE_LAGRANGIAN) return SALE_EINVAL;
  if (!isfinite(c->c_hg) || !(c->c_hg >= 0.0)) return SALE_EINVAL;
  if (c->mode == SALE_LAGRANGIAN && (c->precision != SALE_FP64 || c->remap_order > 1)) return SALE_EINVAL;
  // the step kernels address each field array with 32-bit byte offsets
  const int64_t nnode = (int64_t)(c->nx + 1) * (c->ny + 1) * (c->nz + 1);
  if (nnode * (int64_t)sizeof(double) >= ((int64_t)1 << 32)) return SALE_EINVAL;
  return SALE_OK;
}

Mesh make_mesh(const sale_config *c) {
  Mesh m;
  m.nx = c->nx;
  m.ny = c->ny;
  m.nz = c->nz;
  for (int a = 0; a < 3; a++) m.lo[a] = c->lo[a];
  m.dx = (c->hi[0] - c->lo[0]) / (double)c->nx;
  m.dy = (c->hi[1] - c->lo[1]) / (double)c->ny;
  m.dz = (c->hi[2] - c->lo[2]) / (double)c->nz;
  m.V0 = m.dx * m.dy * m.dz;
  m.iV0 = 1.0 / m.V0;
  m.h = fmin(m.dx, fmin(m.dy, m.dz));
  m.ax = m.dy * m.dz / 4.0;
  m.ay = m.dz * m.dx / 4.0;
  m.az = m.dx * m.dy / 4.0;
  m.gamma = c->gamma;
  m.cfl = c->cfl;
  m.cq = c->c_quad;
  m.cl = c->c_lin;
  m.gm1 = m.gamma - 1.0;
  m.ggm1 = m.gamma * (m.gamma - 1.0);
  m.cq4h = 4.0 * m.cq * m.h;
  m.hyz = m.dy * m.dz;
  m.hzx = m.dz * m.dx;
  m.hxy = m.dx * m.dy;
  m.edx = 0.125 * m.dx;
  m.edy = 0.125 * m.dy;
  m.edz = 0.125 * m.dz;
  m.ncell = (int64_t)c->nx * c->ny * c->nz;
  m.order = c->remap_order == 2 ? 2 : 1;
  m.mode = c->mode == SALE_LAGRANGIAN ? 1 : 0;
  m.chg = c->c_hg;
  m.nnode = (int64_t)(c->nx + 1) * (c->ny + 1) * (c->nz + 1);
  return m;
}

size_t ws_bytes_for(const Mesh &m, int precision) {
  return precision == SALE_FP64 ? sale::workspace_bytes<double>(m) : sale::workspace_bytes<float>(m);
}

int validate_problem(const sale_problem *p, const Mesh &m) {
  if (!p) return SALE_EINVAL;
  if (!isfinite(p->t0) || p->step0 < 0) return SALE_EINVAL;
  switch (p->kind) {
    case SALE_SOD_X:
      if (!isfinite(p->sod[0]) || !finite_pos(p->sod[1]) || !finite_pos(p->sod[2]) ||
          !finite_pos(p->sod[3]) || !finite_pos(p->sod[4]))
        return SALE_EINVAL;
      return SALE_OK;
    case SALE_SEDOV_CORNER:
      if (!finite_pos(p->sedov[0]) || !isfinite(p->sedov[1]) || !(p->sedov[1] >= 0.0) ||
          !isfinite(p->sedov[2]) || !(p->sedov[2] >= 0.0))
        return SALE_EINVAL;
      return SALE_OK;
    case SALE_NOH:
      if (!finite_pos(p->noh[0]) || !isfinite(p->noh[1]) || !(p->noh[1] >= 0.0) || !isfinite(p->noh[2]) ||
          p->noh_dims < 1 || p->noh_dims > 3)
        return SALE_EINVAL;
      return SALE_OK;
    case SALE_USER: {
      if (!p->rho || !p->e || !p->u || !p->v || !p->w) return SALE_EINVAL;
      if (p->user_on_device) return SALE_OK;  // checked on the device at init
      for (int64_t c = 0; c < m.ncell; c++)
        if (!finite_pos(p->rho[c]) || !isfinite(p->e[c]) || !(p->e[c] >= 0.0)) return SALE_EINVAL;
      for (int64_t n = 0; n < m.nnode; n++)
        if (!isfinite(p->u[n]) || !isfinite(p->v[n]) || !isfinite(p->w[n])) return SALE_EINVAL;
      return SALE_OK;
    }
    default:
      return SALE_EINVAL;
  }
}

template <typename R>
hipError_t init_problem(const Mesh &m, Ctl *ctl, const Work<R> &w, const sale_problem *p, double t_end,
                        hipStream_t s) {
  switch (p->kind) {
    case SALE_SOD_X:
      return sale::launch_init_sod<R>(m, ctl, w, p->sod, p->t0, p->step0, t_end, s);
    case SALE_SEDOV_CORNER:
      return sale::launch_init_sedov<R>(m, ctl, w, p->sedov, p->t0, p->step0, t_end, s);
    case SALE_NOH:
      return sale::launch_init_noh<R>(m, ctl, w, p->noh, p->noh_dims, p->t0, p->step0, t_end, s);
    default: {
      const double *const src[5] = {p->rho, p->e, p->u, p->v, p->w};
      return sale::launch_init_user<R>(m, ctl, w, src, p->user_on_device != 0, p->t0, p->step0, t_end, s);
    }
  }
}

int read_ctl(hipStream_t s, const Ctl *d, Ctl *out) {
  hipError_t e = hipMemcpyAsync(out, d, sizeof(Ctl), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e == hipSuccess ? SALE_OK : hip_fail(e, "read control block");
}

int status_code(const Ctl &c) {
  if (c.status & SALE_FLAG_TANGLE) return SALE_ETANGLE;
  if (c.status & SALE_FLAG_NUMERIC) return SALE_ENUMERIC;
  return c.t >= c.t_end ? SALE_DONE : SALE_OK;
}

double next_dt(const Ctl &c, const Mesh &m) {
  double amax = 0.0;
  memcpy(&amax, &c.amax_bits, sizeof(amax));
  const double rem = c.t_end - c.t;
  // the Lagrangian mode keeps the largest a / h of its cells, not of a
  double dt = amax > 0.0 ? (m.mode == 1 ? m.cfl / amax : m.cfl * m.h / amax) : rem;
  return dt > rem ? rem : dt;
}

// Enqueue one step from state buffer `cur` into the other one. A no-op step
// (after t_end or an error) copies the state across, so the current state is
// always in buffer `cur` as the host counts it.
hipError_t enqueue_step(sale_ctx *x) {
  hipError_t e = x->precision == SALE_FP64 ? sale::launch_step<double>(x->m, x->ctl, x->w64, x->cur, x->L, x->stream)
                                           : sale::launch_step<float>(x->m, x->ctl, x->w32, x->cur, x->L, x->stream);
  if (e == hipSuccess) x->cur ^= 1;
  return e;
}

// The graph of kGraphSteps steps starting from state buffer `par`, captured on
// first use. The step kernels take every run-time quantity (dt, t, the done
// decision) from the control block, so one capture serves every replay.
hipError_t step_graph(sale_ctx *x, int par, hipGraphExec_t *out) {
  if (!x->graph[par]) {
    hipError_t e = hipSuccess;
    if (!x->cap_stream) e = hipStreamCreateWithFlags(&x->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    e = hipStreamBeginCapture(x->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t le = hipSuccess;
    for (int s = 0; s < kGraphSteps && le == hipSuccess; s++)
      le = x->precision == SALE_FP64 ? sale::launch_step<double>(x->m, x->ctl, x->w64, par ^ (s & 1), x->L, x->cap_stream)
                                     : sale::launch_step<float>(x->m, x->ctl, x->w32, par ^ (s & 1), x->L, x->cap_stream);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(x->cap_stream, &g);
    if (le != hipSuccess) e = le;
    if (e == hipSuccess) e = hipGraphInstantiate(&x->graph[par], g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      x->graph[par] = nullptr;
      return e;
    }
  }
  *out = x->graph[par];
  return hipSuccess;
}

// n steps on the context's stream: whole graphs, then single steps (only
// single steps while the context is young).
hipError_t enqueue_steps(sale_ctx *x, int64_t n) {
  const bool graphs = x->enqueued >= kGraphAfter && !x->is_static;
  x->enqueued += n;
  for (; graphs && n >= kGraphSteps; n -= kGraphSteps) {
    hipGraphExec_t g;
    hipError_t e = step_graph(x, x->cur, &g);
    if (e == hipSuccess) e = hipGraphLaunch(g, x->stream);
    if (e != hipSuccess) return e;
  }
  for (; n > 0; n--) {
    hipError_t e = enqueue_step(x);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Field export shared by single runs and pool slots (see sale_fields).
int fields_impl(const Mesh &m, int precision, const Work<double> &w64, const Work<float> &w32, int cur,
                Ctl *ctl, hipStream_t stream, uint32_t mask, void *const *dst, int dst_on_device,
                int as_fp64) {
  if (mask && !dst) return SALE_EINVAL;
  if (mask & ~((SALE_F_Z << 1) - 1u)) return SALE_EINVAL;
  if ((mask & SALE_F_Q) && m.mode == 1) return SALE_EINVAL;
  const hipMemcpyKind kind = dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  const bool fp64 = precision == SALE_FP64;
  double *scratch = fp64 ? w64.scratch : w32.scratch;
#define HIP_TRY_F(expr)                               \
  do {                                                \
    hipError_t e_ = (expr);                           \
    if (e_ != hipSuccess) return hip_fail(e_, #expr); \
  } while (0)
  int slot = 0;
  for (uint32_t bit = 1; bit <= SALE_F_Z; bit <<= 1) {
    if (!(mask & bit)) continue;
    void *d = dst[slot++];
    if (!d) return SALE_EINVAL;
    int which = -1;
    switch (bit) {
      case SALE_F_RHO: which = 0; break;
      case SALE_F_E: which = 1; break;
      case SALE_F_P: which = 2; break;
      case SALE_F_Q: which = 3; break;
      case SALE_F_U: which = 4; break;
      case SALE_F_V: which = 5; break;
      case SALE_F_W: which = 6; break;
      default: break;
    }
    if (which >= 0) {
      const int64_t n = which >= 4 ? m.nnode : m.ncell;
      const bool derived = which == 2 || which == 3;
      if (!derived && (fp64 || !as_fp64)) {  // a stored array, copied as is
        const void *src;
        size_t esz;
        if (fp64) {
          const sale::State<double> &st = w64.s[cur];
          const double *arr[7] = {st.rho, st.e, nullptr, nullptr, st.u, st.v, st.w};
          src = arr[which];
          esz = sizeof(double);
        } else {
          const sale::State<float> &st = w32.s[cur];
          const float *arr[7] = {st.rho, st.e, nullptr, nullptr, st.u, st.v, st.w};
          src = arr[which];
          esz = sizeof(float);
        }
        HIP_TRY_F(hipMemcpyAsync(d, src, (size_t)n * esz, kind, stream));
      } else {  // widened or derived: through the scratch array (always double)
        HIP_TRY_F(fp64 ? sale::launch_export<double>(m, w64, cur, which, scratch, stream)
                       : sale::launch_export<float>(m, w32, cur, which, scratch, stream));
        HIP_TRY_F(hipMemcpyAsync(d, scratch, (size_t)n * sizeof(double), kind, stream));
        HIP_TRY_F(hipStreamSynchronize(stream));  // the scratch array is reused next
      }
    } else if (bit == SALE_F_STATE) {
      Ctl c;
      int rc = read_ctl(stream, ctl, &c);
      if (rc != SALE_OK) return rc;
      double *o = (double *)d;
      o[0] = c.t;
      o[1] = (double)c.step;
      o[2] = next_dt(c, m);
      o[3] = (double)c.status;
    } else if (bit == SALE_F_TOTALS) {
      HIP_TRY_F(fp64 ? sale::launch_totals<double>(m, ctl, w64, cur, stream)
                     : sale::launch_totals<float>(m, ctl, w32, cur, stream));
      Ctl c;
      int rc = read_ctl(stream, ctl, &c);
      if (rc != SALE_OK) return rc;
      ((double *)d)[0] = c.totals[0];
      ((double *)d)[1] = c.totals[1];
    } else if (bit == SALE_F_X || bit == SALE_F_Y || bit == SALE_F_Z) {
      const int axis = bit == SALE_F_X ? 0 : bit == SALE_F_Y ? 1 : 2;
      HIP_TRY_F(fp64 ? sale::launch_positions<double>(m, w64, cur, axis, scratch, stream)
                     : sale::launch_positions<float>(m, w32, cur, axis, scratch, stream));
      HIP_TRY_F(hipMemcpyAsync(d, scratch, (size_t)m.nnode * sizeof(double), kind, stream));
      HIP_TRY_F(hipStreamSynchronize(stream));  // the scratch array is reused next
    } else if (bit == SALE_F_CLOCK) {
      Ctl c;
      int rc = read_ctl(stream, ctl, &c);
      if (rc != SALE_OK) return rc;
      int dev = 0, khz = 0;
      HIP_TRY_F(hipGetDevice(&dev));
      HIP_TRY_F(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
      const double hz = khz > 0 ? 1e3 * khz : 1e8;
      ((double *)d)[0] = (double)c.clk_first / hz;
      ((double *)d)[1] = (double)c.clk_last / hz;
    }
  }
  HIP_TRY_F(hipStreamSynchronize(stream));
#undef HIP_TRY_F
  return SALE_OK;
}

// Set up context x (fresh) on the state part `state` and the intermediates
// `inter` (validated config and problem), and enqueue the initial state.
int init_ctx(sale_ctx *x, const sale_config *cfg, const sale_problem *prob, const Mesh &m, void *state,
             void *inter, void *hip_stream) {
  x->cfg = *cfg;
  x->m = m;
  // a mesh at most 3 cells across in y fits one row of 7-row remap tiles,
  // whose 4-wave blocks pass their barriers sooner
  if (m.ny <= 3) x->L.rows_b = 7;
  x->stream = (hipStream_t)hip_stream;
  x->ws = state;
  x->ws_bytes = 0;
  x->t_end = cfg->t_end;
  x->precision = cfg->precision;
  x->cur = 0;
  hipError_t e;
  if (x->precision == SALE_FP64) {
    sale::layout_split<double>(m, state, inter, &x->ctl, &x->w64);
    e = init_problem<double>(m, x->ctl, x->w64, prob, x->t_end, x->stream);
    if (e == hipSuccess && m.mode == 1) e = sale::launch_lag_init(m, x->ctl, x->w64, x->stream);
  } else {
    sale::layout_split<float>(m, state, inter, &x->ctl, &x->w32);
    e = init_problem<float>(m, x->ctl, x->w32, prob, x->t_end, x->stream);
  }
  return e == hipSuccess ? SALE_OK : hip_fail(e, "sale_init");
}

// Host storage of the sale_init_static contexts: one per device, built in
// place (no allocation), released by sale_destroy or by the next
// sale_init_static on the same device.
constexpr int kMaxStaticDevices = 64;
alignas(sale_ctx) unsigned char g_static_mem[kMaxStaticDevices][sizeof(sale_ctx)];
sale_ctx *g_static_ctx[kMaxStaticDevices];
std::mutex g_static_mu;

void release_static(sale_ctx *x) {
  std::lock_guard<std::mutex> lock(g_static_mu);
  for (int d = 0; d < kMaxStaticDevices; d++)
    if (g_static_ctx[d] == x) {
      x->~sale_ctx();
      g_static_ctx[d] = nullptr;
    }
}

}  // namespace sale_host

using namespace sale_host;

#define HIP_TRY(expr)                                 \
  do {                                                \
    hipError_t e_ = (expr);                           \
    if (e_ != hipSuccess) return hip_fail(e_, #expr); \
  } while (0)

extern "C" {

int sale_workspace_bytes(const sale_config *cfg, size_t *bytes) {
  if (!bytes) return SALE_EINVAL;
  int rc = validate_config(cfg);
  if (rc != SALE_OK) return rc;
  *bytes = ws_bytes_for(make_mesh(cfg), cfg->precision);
  return SALE_OK;
}

int sale_init(const sale_config *cfg, const sale_problem *prob, void *d_ws, size_t ws_bytes,
              void *hip_stream, sale_ctx **out) {
  if (!out) return SALE_EINVAL;
  *out = nullptr;
  int rc = validate_config(cfg);
  if (rc != SALE_OK) return rc;
  Mesh m = make_mesh(cfg);
  if ((rc = validate_problem(prob, m)) != SALE_OK) return rc;
  if (!d_ws || ((uintptr_t)d_ws & 255u)) return SALE_EINVAL;
  if (ws_bytes < ws_bytes_for(m, cfg->precision)) return SALE_ENOMEM;
  sale_ctx *x = new (std::nothrow) sale_ctx;
  if (!x) return SALE_ENOMEM;
  const size_t sb = cfg->precision == SALE_FP64 ? sale::state_bytes<double>(m) : sale::state_bytes<float>(m);
  if ((rc = init_ctx(x, cfg, prob, m, d_ws, (char *)d_ws + sb, hip_stream)) != SALE_OK) {
    delete x;
    return rc;
  }
  *out = x;
  return SALE_OK;
}

int sale_init_static(const sale_config *cfg, const sale_problem *prob, void *d_state, size_t *state_bytes,
                     void *hip_stream, sale_ctx **out) {
  if (!state_bytes) return SALE_EINVAL;
  if (out) *out = nullptr;
  int rc = validate_config(cfg);
  if (rc != SALE_OK) return rc;
  const Mesh m = make_mesh(cfg);
  const bool fp64 = cfg->precision == SALE_FP64;
  const size_t need = fp64 ? sale::state_bytes<double>(m) : sale::state_bytes<float>(m);
  const size_t inter = fp64 ? sale::inter_bytes<double>(m) : sale::inter_bytes<float>(m);
  if (inter > sale::kStaticScratchBytes) return SALE_ENOMEM;  // beyond the library's device array
  if (!d_state) {  // size query
    *state_bytes = need;
    return SALE_OK;
  }
  if (!out) return SALE_EINVAL;
  if ((rc = validate_problem(prob, m)) != SALE_OK) return rc;
  if (((uintptr_t)d_state & 255u)) return SALE_EINVAL;
  if (*state_bytes < need) return SALE_ENOMEM;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxStaticDevices) return SALE_EINVAL;
  void *scr = nullptr;
  HIP_TRY(sale::static_scratch(&scr));
  std::lock_guard<std::mutex> lock(g_static_mu);
  sale_ctx *x = g_static_ctx[dev];
  if (x) {  // the device's previous static context ends here
    x->~sale_ctx();
    g_static_ctx[dev] = nullptr;
  }
  x = new (g_static_mem[dev]) sale_ctx;
  x->is_static = true;
  if ((rc = init_ctx(x, cfg, prob, m, d_state, scr, hip_stream)) != SALE_OK) {
    x->~sale_ctx();
    return rc;
  }
  g_static_ctx[dev] = x;
  *out = x;
  return SALE_OK;
}

int sale_step(sale_ctx *x) {
  if (!x) return SALE_EINVAL;
  HIP_TRY(enqueue_step(x));
  return SALE_OK;
}

int sale_run(sale_ctx *x, double t_end, int64_t max_steps) {
  if (!x || max_steps < 0) return SALE_EINVAL;
  if (isnan(t_end)) return SALE_EINVAL;
  if (t_end >= 0.0) {
    x->t_end = t_end;
    HIP_TRY(sale::launch_set_t_end(x->ctl, t_end, x->stream));
  }
  Ctl c;
  int rc = read_ctl(x->stream, x->ctl, &c);
  if (rc != SALE_OK) return rc;
  if ((rc = status_code(c)) != SALE_OK) return rc;
  int64_t left = max_steps;
  long long last_step = c.step;
  double last_t = c.t;
  int64_t chunk = 4;
  while (left > 0) {
    const int64_t n = std::min(left, chunk);
    HIP_TRY(enqueue_steps(x, n));
    left -= n;
    if ((rc = read_ctl(x->stream, x->ctl, &c)) != SALE_OK) return rc;
    if ((rc = status_code(c)) != SALE_OK) return rc;
    // size the next chunk from the observed step rate, so that few enqueued
    // steps land past t_end (those are no-ops)
    const long long took = c.step - last_step;
    if (took > 0 && c.t > last_t) {
      const double per = (c.t - last_t) / (double)took;
      const double est = (c.t_end - c.t) / per;
      chunk = (int64_t)std::max(1.0, std::min(256.0, 0.9 * est));
      if (chunk >= kGraphSteps) chunk -= chunk % kGraphSteps;  // whole graphs
    }
    last_step = c.step;
    last_t = c.t;
  }
  return SALE_OK;
}

int sale_status(sale_ctx *x, int32_t *flags) {
  if (!x) return SALE_EINVAL;
  Ctl c;
  int rc = read_ctl(x->stream, x->ctl, &c);
  if (rc != SALE_OK) return rc;
  if (flags) *flags = (int32_t)c.status;
  return status_code(c);
}

int sale_fields(sale_ctx *x, uint32_t mask, void *const *dst, int dst_on_device, int as_fp64) {
  if (!x) return SALE_EINVAL;
  return fields_impl(x->m, x->precision, x->w64, x->w32, x->cur, x->ctl, x->stream, mask, dst, dst_on_device,
                     as_fp64);
}

void sale_destroy(sale_ctx *x) {
  if (x && x->is_static)
    sale_host::release_static(x);
  else
    delete x;
}

const char *sale_strerror(int code) {
  switch (code) {
    case SALE_OK: return "ok";
    case SALE_DONE: return "run complete (t >= t_end)";
    case SALE_EINVAL: return "invalid argument, configuration or initial data";
    case SALE_ENOMEM: return "workspace or arena too small";
    case SALE_EHIP: return g_hip_msg;
    case SALE_ENUMERIC: return "numeric failure: non-positive density, negative energy or non-finite value";
    case SALE_ETANGLE: return "tangled cell: predictor or Lagrangian volume <= 0";
    case SALE_EBUSY: return "admission refused: no free slot or over the memory budget";
    default: return "unknown code";
  }
}

}  // extern "C"

// =====================================================================================
// pool
// =====================================================================================
#include <vector>

namespace sale_host {

struct PoolSlot {
  bool used = false;
  bool reported = false;  // listed by a poll as finished
  size_t off = 0, bytes = 0;
  Mesh m;
  Work<double> w64;
  Work<float> w32;
  Ctl *ctl = nullptr;  // in the pool header
  long long step0 = 0;
  long long step_target = 0;
  int nA = 0, nB = 0;
  sale::PoolRun<double> r64;  // host images of the device slot entry
  sale::PoolRun<float> r32;
};

}  // namespace sale_host

struct sale_pool {
  int precision;
  int max_runs;
  char *arena;
  size_t arena_bytes;
  hipStream_t stream;
  size_t hdr_bytes;
  sale::PoolQueue *d_q;
  void *d_runs;
  Ctl *d_ctl;
  int *d_act, *d_prefA, *d_prefB;
  std::vector<sale_host::PoolSlot> slots;
  std::vector<std::pair<size_t, size_t>> free_list;  // (offset, size), sorted, disjoint
  std::vector<int> h_act, h_prefA, h_prefB;
  std::vector<Ctl> h_ctl;
  sale::PoolQueue h_q = {};
  int resident;
  // advance mode: 0 chosen per advance, 1 always the persistent kernel, 2
  // always lockstep launches (SALE_POOL_PERSISTENT unset, 1, 0)
  int mode = 0;
  // With SALE_POOL_GRAPHS=1 at creation, lockstep rounds after an advance's
  // first are replays of one captured graph of a round (its four launches),
  // kept while the round's shape -- active runs and block counts -- stays
  // the same; by default every round is launched.
  bool graphs = false;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t round_graph = nullptr;
  int g_nact = -1, g_totA = -1, g_totB = -1;
  // XCD ids of the device (bit g: XCD g), from a probe launch at the first
  // persistent advance, or SALE_POOL_XCC_MASK at sale_pool_create
  unsigned int xcc_mask = 0;
  bool xcc_known = false;
  // cap of one wait of the persistent kernel, in ticks of the 100 MHz device
  // clock (2 s; SALE_POOL_WAIT_TICKS at creation, a test hook)
  long long wait_ticks = 200000000ll;
  ~sale_pool() {
    if (round_graph) {
      (void)hipStreamSynchronize(stream);  // replays of it may still be queued
      (void)hipGraphExecDestroy(round_graph);
    }
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
  }
};

namespace sale_host {

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

bool pool_alloc(sale_pool *p, size_t bytes, size_t *off) {
  for (size_t k = 0; k < p->free_list.size(); k++) {
    auto &fr = p->free_list[k];
    if (fr.second >= bytes) {
      *off = fr.first;
      fr.first += bytes;
      fr.second -= bytes;
      if (fr.second == 0) p->free_list.erase(p->free_list.begin() + k);
      return true;
    }
  }
  return false;
}

void pool_free(sale_pool *p, size_t off, size_t bytes) {
  auto &fl = p->free_list;
  size_t k = 0;
  while (k < fl.size() && fl[k].first < off) k++;
  fl.insert(fl.begin() + k, {off, bytes});
  if (k + 1 < fl.size() && fl[k].first + fl[k].second == fl[k + 1].first) {  // merge right
    fl[k].second += fl[k + 1].second;
    fl.erase(fl.begin() + k + 1);
  }
  if (k > 0 && fl[k - 1].first + fl[k - 1].second == fl[k].first) {  // merge left
    fl[k - 1].second += fl[k].second;
    fl.erase(fl.begin() + k);
  }
}

template <typename R>
sale::PoolRun<R> pool_image(const PoolSlot &sl, const Work<R> &w) {
  sale::PoolRun<R> r;
  r.m = sl.m;
  r.ctl = sl.ctl;
  r.s[0] = w.s[0];
  r.s[1] = w.s[1];
  r.up = w.up;
  r.vp = w.vp;
  r.wp = w.wp;
  r.geo = w.geo;
  // one z segment per tile: the pool's parallelism comes from its many runs
  r.ga = sale::grid_lagrange(sl.m, 1, sale::kPoolRows, sale::kPoolWidth);
  r.gb = sale::grid_remap(sl.m, 1, sale::kPoolRows, sale::kPoolWidth);
  r.step0 = sl.step0;
  r.step_target = sl.step_target;
  return r;
}

bool finished(const Ctl &c, long long step_target) {
  return c.status != 0u || c.t >= c.t_end || c.step >= step_target;
}

}  // namespace sale_host

extern "C" {

int sale_pool_create(int32_t precision, int32_t max_runs, void *d_arena, size_t arena_bytes, void *hip_stream,
                     sale_pool **out) {
  if (!out) return SALE_EINVAL;
  *out = nullptr;
  if ((precision != SALE_FP64 && precision != SALE_MIXED32) || max_runs < 1 || max_runs > (1 << 20))
    return SALE_EINVAL;
  if (!d_arena || ((uintptr_t)d_arena & 255u)) return SALE_EINVAL;
  const size_t run_sz = precision == SALE_FP64 ? sizeof(sale::PoolRun<double>) : sizeof(sale::PoolRun<float>);
  size_t hdr = a256(sizeof(sale::PoolQueue)) + a256((size_t)max_runs * run_sz) + a256((size_t)max_runs * sizeof(Ctl)) +
               3 * a256((size_t)(max_runs + 1) * sizeof(int));
  if (arena_bytes < hdr) return SALE_ENOMEM;
  sale_pool *p = new (std::nothrow) sale_pool;
  if (!p) return SALE_ENOMEM;
  p->precision = precision;
  p->max_runs = max_runs;
  p->arena = (char *)d_arena;
  p->arena_bytes = arena_bytes;
  p->stream = (hipStream_t)hip_stream;
  p->hdr_bytes = hdr;
  char *q = p->arena;
  p->d_q = (sale::PoolQueue *)q;
  q += a256(sizeof(sale::PoolQueue));
  p->d_runs = q;
  q += a256((size_t)max_runs * run_sz);
  p->d_ctl = (Ctl *)q;
  q += a256((size_t)max_runs * sizeof(Ctl));
  p->d_act = (int *)q;
  q += a256((size_t)(max_runs + 1) * sizeof(int));
  p->d_prefA = (int *)q;
  q += a256((size_t)(max_runs + 1) * sizeof(int));
  p->d_prefB = (int *)q;
  p->slots.resize(max_runs);
  p->free_list.push_back({hdr, arena_bytes - hdr});
  p->h_ctl.resize(max_runs);
  p->resident = precision == SALE_FP64 ? sale::pool_resident_blocks<double>() : sale::pool_resident_blocks<float>();
  // SALE_POOL_PERSISTENT=1 / 0: every advance by the persistent kernel / by
  // lockstep launches; unset: chosen per advance
  const char *pers = getenv("SALE_POOL_PERSISTENT");
  p->mode = pers && pers[0] == '1' ? 1 : pers && pers[0] == '0' ? 2 : 0;
  const char *gr = getenv("SALE_POOL_GRAPHS");
  p->graphs = gr && gr[0] == '1';
  // SALE_POOL_XCC_MASK: the XCDs the persistent advance assigns runs to,
  // instead of the probed ones (a test hook: a run on an XCD that serves no
  // block is flagged, not advanced)
  const char *wt = getenv("SALE_POOL_WAIT_TICKS");
  if (wt && wt[0]) p->wait_ticks = std::max(0ll, strtoll(wt, nullptr, 0));
  const char *xm = getenv("SALE_POOL_XCC_MASK");
  if (xm && xm[0]) {
    p->xcc_mask = (unsigned int)strtoul(xm, nullptr, 0) & ((1u << sale::kPoolGroups) - 1u);
    p->xcc_known = p->xcc_mask != 0;
  }
  *out = p;
  return SALE_OK;
}

int sale_pool_admit(sale_pool *p, const sale_config *cfg, const sale_problem *prob, int64_t n_steps,
                    int32_t *slot) {
  if (!p || !slot || n_steps < 0) return SALE_EINVAL;
  int rc = validate_config(cfg);
  if (rc != SALE_OK) return rc;
  if (cfg->precision != p->precision) return SALE_EINVAL;
  const Mesh m = make_mesh(cfg);
  if (m.order != 1 || m.mode != 0) return SALE_EINVAL;  // the persistent kernel: Eulerian, first order
  if ((rc = validate_problem(prob, m)) != SALE_OK) return rc;
  const size_t bytes = a256(ws_bytes_for(m, p->precision));
  if (bytes > p->arena_bytes - p->hdr_bytes) return SALE_ENOMEM;  // would never fit
  int s = -1;
  for (int k = 0; k < p->max_runs; k++)
    if (!p->slots[k].used) {
      s = k;
      break;
    }
  if (s < 0) return SALE_EBUSY;
  size_t off;
  if (!pool_alloc(p, bytes, &off)) return SALE_EBUSY;
  PoolSlot &sl = p->slots[s];
  sl.off = off;
  sl.bytes = bytes;
  sl.m = m;
  sl.ctl = p->d_ctl + s;
  sl.step0 = prob->step0;
  sl.step_target = prob->step0 + n_steps;
  sl.reported = false;
  Ctl *unused;
  hipError_t e;
  if (p->precision == SALE_FP64) {
    sale::layout<double>(m, p->arena + off, &unused, &sl.w64);
    e = init_problem<double>(m, sl.ctl, sl.w64, prob, cfg->t_end, p->stream);
    sl.r64 = pool_image<double>(sl, sl.w64);
    sl.nA = sl.r64.ga.blocks();
    sl.nB = sl.r64.gb.blocks();
    if (e == hipSuccess)
      e = hipMemcpyAsync((sale::PoolRun<double> *)p->d_runs + s, &sl.r64, sizeof(sl.r64), hipMemcpyHostToDevice,
                         p->stream);
  } else {
    sale::layout<float>(m, p->arena + off, &unused, &sl.w32);
    e = init_problem<float>(m, sl.ctl, sl.w32, prob, cfg->t_end, p->stream);
    sl.r32 = pool_image<float>(sl, sl.w32);
    sl.nA = sl.r32.ga.blocks();
    sl.nB = sl.r32.gb.blocks();
    if (e == hipSuccess)
      e = hipMemcpyAsync((sale::PoolRun<float> *)p->d_runs + s, &sl.r32, sizeof(sl.r32), hipMemcpyHostToDevice,
                         p->stream);
  }
  // the host images are read by the copy above: keep them unchanged until it ran
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) {
    pool_free(p, off, bytes);
    return hip_fail(e, "sale_pool_admit");
  }
  sl.used = true;
  *slot = s;
  return SALE_OK;
}

int sale_pool_advance(sale_pool *p, int32_t max_steps_per_run) {
  if (!p || max_steps_per_run < 0) return SALE_EINVAL;
  if (max_steps_per_run == 0) return SALE_OK;
  // the host tables of the previous advance may still be in a copy: wait
  hipError_t e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return hip_fail(e, "sale_pool_advance");
  p->h_act.clear();
  p->h_prefA.assign(1, 0);
  p->h_prefB.assign(1, 0);
  for (int k = 0; k < p->max_runs; k++) {
    const PoolSlot &sl = p->slots[k];
    if (!sl.used || sl.reported) continue;
    p->h_act.push_back(k);
    p->h_prefA.push_back(p->h_prefA.back() + sl.nA);
    p->h_prefB.push_back(p->h_prefB.back() + sl.nB);
  }
  const int nact = (int)p->h_act.size();
  if (nact == 0) return SALE_OK;
  // The persistent kernel serves each run from the blocks of one XCD: one
  // group of runs per XCD, balanced by cells (largest first, each to the least
  // loaded XCD). Chosen per advance: the persistent kernel when there are at
  // least four runs per XCD and the busiest is within 10% of the mean load, else
  // lockstep launches (few or uneven runs leave XCDs idle in the persistent
  // kernel).
  bool persistent = p->mode == 1;
  std::vector<int> grp(p->max_runs, -1);
  if (p->mode != 2) {
    if (!p->xcc_known) {
      unsigned int mask = 0;
      HIP_TRY(hipMemsetAsync(&p->d_q->xcc_mask, 0, sizeof(unsigned int), p->stream));
      HIP_TRY(sale::launch_xcc_probe(p->d_q, p->stream));
      HIP_TRY(hipMemcpyAsync(&mask, &p->d_q->xcc_mask, sizeof(unsigned int), hipMemcpyDeviceToHost, p->stream));
      HIP_TRY(hipStreamSynchronize(p->stream));
      if (mask == 0) return SALE_EHIP;
      p->xcc_mask = mask;
      p->xcc_known = true;
    }
    std::vector<int> order = p->h_act;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return p->slots[a].m.ncell > p->slots[b].m.ncell; });
    double load[sale::kPoolGroups] = {}, total = 0.0;
    int nx = 0;
    for (int g = 0; g < sale::kPoolGroups; g++) nx += (int)(p->xcc_mask >> g & 1u);
    for (int k : order) {
      int best = -1;
      for (int g = 0; g < sale::kPoolGroups; g++)
        if ((p->xcc_mask >> g & 1u) && (best < 0 || load[g] < load[best])) best = g;
      grp[k] = best;
      load[best] += (double)p->slots[k].m.ncell;
      total += (double)p->slots[k].m.ncell;
    }
    const double busiest = *std::max_element(load, load + sale::kPoolGroups);
    if (p->mode == 0) persistent = nact >= 4 * nx && busiest <= 1.1 * total / nx;
  }
  {
    // z split of each run sized to its share of the advance's cells, about
    // `target` tiles per phase in all (one segment for runs too small, and
    // for every run when the target is 0)
    const double target = persistent ? (double)SALE_POOL_PERSISTENT_BLOCKS : 3072.0;
    double cells = 0.0;
    for (int k : p->h_act) cells += (double)p->slots[k].m.ncell;
    if (persistent) {
      // act lists the XCD groups in XCD order, each in slot order
      std::vector<int> act;
      for (int g = 0; g < sale::kPoolGroups; g++) {
        p->h_q.gact[g] = (int)act.size();
        for (int k : p->h_act)
          if (grp[k] == g) act.push_back(k);
      }
      p->h_q.gact[sale::kPoolGroups] = (int)act.size();
      p->h_act = act;
    }
    p->h_prefA.assign(1, 0);
    p->h_prefB.assign(1, 0);
    for (int k : p->h_act) {
      PoolSlot &sl = p->slots[k];
      const int quota = (int)std::max(1.0, target * (double)sl.m.ncell / cells);
      const sale::Grid2 ga = sale::grid_lagrange(sl.m, quota, sale::kPoolRows, sale::kPoolWidth);
      const sale::Grid2 gb = sale::grid_remap(sl.m, quota, sale::kPoolRows, sale::kPoolWidth);
      hipError_t ce;
      if (p->precision == SALE_FP64) {
        sl.r64.ga = ga, sl.r64.gb = gb;
        ce = hipMemcpyAsync((sale::PoolRun<double> *)p->d_runs + k, &sl.r64, sizeof(sl.r64), hipMemcpyHostToDevice,
                            p->stream);
      } else {
        sl.r32.ga = ga, sl.r32.gb = gb;
        ce = hipMemcpyAsync((sale::PoolRun<float> *)p->d_runs + k, &sl.r32, sizeof(sl.r32), hipMemcpyHostToDevice,
                            p->stream);
      }
      if (ce != hipSuccess) return hip_fail(ce, "sale_pool_advance");
      p->h_prefA.push_back(p->h_prefA.back() + ga.blocks());
      p->h_prefB.push_back(p->h_prefB.back() + gb.blocks());
    }
  }
  const int totA = p->h_prefA.back(), totB = p->h_prefB.back();
  HIP_TRY(hipMemcpyAsync(p->d_act, p->h_act.data(), nact * sizeof(int), hipMemcpyHostToDevice, p->stream));
  HIP_TRY(hipMemcpyAsync(p->d_prefA, p->h_prefA.data(), (nact + 1) * sizeof(int), hipMemcpyHostToDevice, p->stream));
  HIP_TRY(hipMemcpyAsync(p->d_prefB, p->h_prefB.data(), (nact + 1) * sizeof(int), hipMemcpyHostToDevice, p->stream));
  if (!persistent) {
    auto rounds = [&](int n, int first, hipStream_t s) {
      return p->precision == SALE_FP64
                 ? sale::launch_pool_lockstep<double>((const sale::PoolRun<double> *)p->d_runs, p->d_act,
                                                      p->d_prefA, p->d_prefB, nact, totA, totB, n, first, s)
                 : sale::launch_pool_lockstep<float>((const sale::PoolRun<float> *)p->d_runs, p->d_act,
                                                     p->d_prefA, p->d_prefB, nact, totA, totB, n, first, s);
    };
    if (!p->graphs || max_steps_per_run < 2) {
      HIP_TRY(rounds(max_steps_per_run, 1, p->stream));
      return SALE_OK;
    }
    HIP_TRY(rounds(1, 1, p->stream));
    if (!p->round_graph || p->g_nact != nact || p->g_totA != totA || p->g_totB != totB) {
      if (p->round_graph) {
        HIP_TRY(hipGraphExecDestroy(p->round_graph));
        p->round_graph = nullptr;
      }
      if (!p->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
      HIP_TRY(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
      const hipError_t le = rounds(1, 0, p->cap_stream);
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamEndCapture(p->cap_stream, &g);
      if (le != hipSuccess) e = le;
      if (e == hipSuccess) e = hipGraphInstantiate(&p->round_graph, g, nullptr, nullptr, 0);
      if (g) (void)hipGraphDestroy(g);
      if (e != hipSuccess) {
        p->round_graph = nullptr;
        return hip_fail(e, "sale_pool_advance (round graph)");
      }
      p->g_nact = nact, p->g_totA = totA, p->g_totB = totB;
    }
    for (int r = 1; r < max_steps_per_run; r++) HIP_TRY(hipGraphLaunch(p->round_graph, p->stream));
    return SALE_OK;
  }
  for (int g = 0; g < sale::kPoolGroups; g++) p->h_q.head[g] = 0;
  p->h_q.nact = nact;
  p->h_q.rounds = max_steps_per_run;
  p->h_q.totA = totA;
  p->h_q.totB = totB;
  p->h_q.wait_ticks = p->wait_ticks;
  p->h_q.timeouts = 0;
  p->h_q.abort = 0;
  p->h_q.exited = 0;
  p->h_q.starved = 0;
  p->h_q.xcc_mask = p->xcc_mask;
  // every resident block, so that every XCD receives blocks (a block whose
  // XCD serves no run leaves at once)
  const int blocks = p->resident;
  HIP_TRY(hipMemcpyAsync(p->d_q, &p->h_q, sizeof(p->h_q), hipMemcpyHostToDevice, p->stream));
  if (p->precision == SALE_FP64)
    HIP_TRY(sale::launch_pool_advance<double>((sale::PoolRun<double> *)p->d_runs, p->d_act, p->d_prefA, p->d_prefB,
                                              p->d_q, nact, blocks, p->stream));
  else
    HIP_TRY(sale::launch_pool_advance<float>((sale::PoolRun<float> *)p->d_runs, p->d_act, p->d_prefA, p->d_prefB,
                                             p->d_q, nact, blocks, p->stream));
  return SALE_OK;
}

int sale_pool_poll(sale_pool *p, int32_t *done, int32_t cap, int32_t *n_done) {
  if (!p || !n_done || cap < 0 || (cap > 0 && !done)) return SALE_EINVAL;
  *n_done = 0;
  HIP_TRY(hipMemcpyAsync(p->h_ctl.data(), p->d_ctl, p->max_runs * sizeof(Ctl), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  for (int k = 0; k < p->max_runs && *n_done < cap; k++) {
    PoolSlot &sl = p->slots[k];
    if (!sl.used || sl.reported) continue;
    if (finished(p->h_ctl[k], sl.step_target)) {
      sl.reported = true;
      done[(*n_done)++] = k;
    }
  }
  return SALE_OK;
}

int sale_pool_fields(sale_pool *p, int32_t slot, uint32_t mask, void *const *dst, int dst_on_device,
                     int as_fp64) {
  if (!p || slot < 0 || slot >= p->max_runs || !p->slots[slot].used) return SALE_EINVAL;
  PoolSlot &sl = p->slots[slot];
  Ctl c;
  int rc = read_ctl(p->stream, sl.ctl, &c);
  if (rc != SALE_OK) return rc;
  const int cur = (int)((c.step - sl.step0) & 1);
  return fields_impl(sl.m, p->precision, sl.w64, sl.w32, cur, sl.ctl, p->stream, mask, dst, dst_on_device,
                     as_fp64);
}

int sale_pool_release(sale_pool *p, int32_t slot) {
  if (!p || slot < 0 || slot >= p->max_runs || !p->slots[slot].used) return SALE_EINVAL;
  HIP_TRY(hipStreamSynchronize(p->stream));
  PoolSlot &sl = p->slots[slot];
  pool_free(p, sl.off, sl.bytes);
  sl.used = false;
  sl.reported = false;
  return SALE_OK;
}

void sale_pool_destroy(sale_pool *p) { delete p; }

}  // extern "C"

extern "C" int sale_step_timed(sale_ctx *x, int32_t n, float ms[3]) {
  if (!x || n < 1 || !ms) return SALE_EINVAL;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  hipError_t e = hipSuccess;
  for (int k = 0; k < 4 && e == hipSuccess; k++) e = hipEventCreate(&ev[k]);
  double acc[3] = {0.0, 0.0, 0.0};
  for (int32_t i = 0; i < n && e == hipSuccess; i++) {
    e = x->precision == SALE_FP64 ? sale::launch_step<double>(x->m, x->ctl, x->w64, x->cur, x->L, x->stream, ev)
                                  : sale::launch_step<float>(x->m, x->ctl, x->w32, x->cur, x->L, x->stream, ev);
    if (e != hipSuccess) break;
    x->cur ^= 1;
    e = hipEventSynchronize(ev[3]);
    for (int k = 0; k < 3 && e == hipSuccess; k++) {
      float t = 0.f;
      e = hipEventElapsedTime(&t, ev[k], ev[k + 1]);
      acc[k] += t;
    }
  }
  for (int k = 0; k < 4; k++)
    if (ev[k]) (void)hipEventDestroy(ev[k]);
  if (e != hipSuccess) return hip_fail(e, "sale_step_timed");
  for (int k = 0; k < 3; k++) ms[k] = (float)acc[k];
  return SALE_OK;
}

extern "C" int sale_set_launch(sale_ctx *x, int32_t rows_lagrange, int32_t rows_remap, int32_t target_blocks) {
  if (!x) return SALE_EINVAL;
  sale::Launch L;
  L.rows_a = rows_lagrange;
  L.rows_b = rows_remap;
  L.target = target_blocks;
  if (!sale::launch_valid(L)) return SALE_EINVAL;
  // captured step graphs hold the old shape; wait for replays in flight first
  HIP_TRY(hipStreamSynchronize(x->stream));
  for (int k = 0; k < 2; k++)
    if (x->graph[k]) {
      (void)hipGraphExecDestroy(x->graph[k]);
      x->graph[k] = nullptr;
    }
  x->L = L;
  return SALE_OK;
}

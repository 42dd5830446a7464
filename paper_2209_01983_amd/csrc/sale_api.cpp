// sale_api.cpp -- host side of the libsale C ABI declared in include/sale.h:
// argument validation, workspace layout, enqueueing of the step kernels on
// the caller's stream, status polling and field export, for both precisions.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>

#include "../../include/sale.h"
#include "sale_impl.h"

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
};

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
  const int64_t ncell = (int64_t)c->nx * c->ny * c->nz;
  if (ncell > ((int64_t)1 << 34)) return SALE_EINVAL;
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
  m.h = fmin(m.dx, fmin(m.dy, m.dz));
  m.ax = m.dy * m.dz / 4.0;
  m.ay = m.dz * m.dx / 4.0;
  m.az = m.dx * m.dy / 4.0;
  m.gamma = c->gamma;
  m.cfl = c->cfl;
  m.cq = c->c_quad;
  m.cl = c->c_lin;
  m.ncell = (int64_t)c->nx * c->ny * c->nz;
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
  double dt = amax > 0.0 ? m.cfl * m.h / amax : rem;
  return dt > rem ? rem : dt;
}

// Enqueue one step from state buffer `cur` into the other one. A no-op step
// (after t_end or an error) copies the state across, so the current state is
// always in buffer `cur` as the host counts it.
hipError_t enqueue_step(sale_ctx *x) {
  hipError_t e = x->precision == SALE_FP64 ? sale::launch_step<double>(x->m, x->ctl, x->w64, x->cur, x->stream)
                                           : sale::launch_step<float>(x->m, x->ctl, x->w32, x->cur, x->stream);
  if (e == hipSuccess) x->cur ^= 1;
  return e;
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
  x->cfg = *cfg;
  x->m = m;
  x->stream = (hipStream_t)hip_stream;
  x->ws = d_ws;
  x->ws_bytes = ws_bytes;
  x->t_end = cfg->t_end;
  x->precision = cfg->precision;
  x->cur = 0;
  hipError_t e;
  if (x->precision == SALE_FP64) {
    sale::layout<double>(m, d_ws, &x->ctl, &x->w64);
    e = init_problem<double>(m, x->ctl, x->w64, prob, x->t_end, x->stream);
  } else {
    sale::layout<float>(m, d_ws, &x->ctl, &x->w32);
    e = init_problem<float>(m, x->ctl, x->w32, prob, x->t_end, x->stream);
  }
  if (e != hipSuccess) {
    delete x;
    return hip_fail(e, "sale_init");
  }
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
    for (int64_t s = 0; s < n; s++) HIP_TRY(enqueue_step(x));
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
  if (!x || (mask && !dst)) return SALE_EINVAL;
  if (mask & ~((SALE_F_TOTALS << 1) - 1u)) return SALE_EINVAL;
  const Mesh &m = x->m;
  const hipMemcpyKind kind = dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  const bool fp64 = x->precision == SALE_FP64;
  double *scratch = fp64 ? x->w64.scratch : x->w32.scratch;
  int slot = 0;
  for (uint32_t bit = 1; bit <= SALE_F_TOTALS; bit <<= 1) {
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
          const sale::State<double> &s = x->w64.s[x->cur];
          const double *arr[7] = {s.rho, s.e, nullptr, nullptr, s.u, s.v, s.w};
          src = arr[which];
          esz = sizeof(double);
        } else {
          const sale::State<float> &s = x->w32.s[x->cur];
          const float *arr[7] = {s.rho, s.e, nullptr, nullptr, s.u, s.v, s.w};
          src = arr[which];
          esz = sizeof(float);
        }
        HIP_TRY(hipMemcpyAsync(d, src, (size_t)n * esz, kind, x->stream));
      } else {  // widened or derived: through the scratch array (always double)
        HIP_TRY(fp64 ? sale::launch_export<double>(m, x->w64, x->cur, which, scratch, x->stream)
                     : sale::launch_export<float>(m, x->w32, x->cur, which, scratch, x->stream));
        HIP_TRY(hipMemcpyAsync(d, scratch, (size_t)n * sizeof(double), kind, x->stream));
        HIP_TRY(hipStreamSynchronize(x->stream));  // the scratch array is reused next
      }
    } else if (bit == SALE_F_STATE) {
      Ctl c;
      int rc = read_ctl(x->stream, x->ctl, &c);
      if (rc != SALE_OK) return rc;
      double *o = (double *)d;
      o[0] = c.t;
      o[1] = (double)c.step;
      o[2] = next_dt(c, m);
      o[3] = (double)c.status;
    } else if (bit == SALE_F_TOTALS) {
      HIP_TRY(fp64 ? sale::launch_totals<double>(m, x->ctl, x->w64, x->cur, x->stream)
                   : sale::launch_totals<float>(m, x->ctl, x->w32, x->cur, x->stream));
      Ctl c;
      int rc = read_ctl(x->stream, x->ctl, &c);
      if (rc != SALE_OK) return rc;
      ((double *)d)[0] = c.totals[0];
      ((double *)d)[1] = c.totals[1];
    }
  }
  HIP_TRY(hipStreamSynchronize(x->stream));
  return SALE_OK;
}

void sale_destroy(sale_ctx *x) { delete x; }

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

// sale_api.cpp -- host side of the libsale C ABI declared in include/sale.h:
// argument validation, workspace layout, enqueueing of the step kernels on
// the caller's stream, status polling and field export.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "../../include/sale.h"
#include "sale_impl.h"

using sale::Ctl;
using sale::Fields64;
using sale::Mesh;

struct sale_ctx {
  sale_config cfg;
  Mesh m;
  hipStream_t stream;
  void *ws;
  size_t ws_bytes;
  Ctl *ctl;
  Fields64 f;
  double t_end;
};

namespace {

thread_local char g_hip_msg[256] = "no HIP error recorded";

int hip_fail(hipError_t e, const char *what) {
  snprintf(g_hip_msg, sizeof(g_hip_msg), "%s: %s", what, hipGetErrorString(e));
  return SALE_EHIP;
}

#define HIP_TRY(expr)                               \
  do {                                              \
    hipError_t e_ = (expr);                         \
    if (e_ != hipSuccess) return hip_fail(e_, #expr); \
  } while (0)

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
  if (c->precision != SALE_FP64) return SALE_EINVAL;  // MIXED32 not in this build
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

int read_ctl(sale_ctx *x, Ctl *out) {
  HIP_TRY(hipMemcpyAsync(out, x->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, x->stream));
  HIP_TRY(hipStreamSynchronize(x->stream));
  return SALE_OK;
}

int status_code(const Ctl &c) {
  if (c.status & SALE_FLAG_TANGLE) return SALE_ETANGLE;
  if (c.status & SALE_FLAG_NUMERIC) return SALE_ENUMERIC;
  return c.t >= c.t_end ? SALE_DONE : SALE_OK;
}

}  // namespace

extern "C" {

int sale_workspace_bytes(const sale_config *cfg, size_t *bytes) {
  if (!bytes) return SALE_EINVAL;
  int rc = validate_config(cfg);
  if (rc != SALE_OK) return rc;
  Mesh m = make_mesh(cfg);
  *bytes = sale::workspace_bytes_fp64(m, nullptr);
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
  if (ws_bytes < sale::workspace_bytes_fp64(m, nullptr)) return SALE_ENOMEM;
  sale_ctx *x = new (std::nothrow) sale_ctx;
  if (!x) return SALE_ENOMEM;
  x->cfg = *cfg;
  x->m = m;
  x->stream = (hipStream_t)hip_stream;
  x->ws = d_ws;
  x->ws_bytes = ws_bytes;
  x->t_end = cfg->t_end;
  sale::layout_fp64(m, d_ws, &x->ctl, &x->f);
  hipError_t e = hipSuccess;
  const double t0 = prob->t0;
  switch (prob->kind) {
    case SALE_SOD_X:
      e = sale::launch_init_sod(m, x->ctl, x->f, prob->sod, t0, prob->step0, x->t_end, x->stream);
      break;
    case SALE_SEDOV_CORNER:
      e = sale::launch_init_sedov(m, x->ctl, x->f, prob->sedov, t0, prob->step0, x->t_end, x->stream);
      break;
    default: {
      const hipMemcpyKind kind = prob->user_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
      const size_t cb = (size_t)m.ncell * sizeof(double), nb = (size_t)m.nnode * sizeof(double);
      if ((e = hipMemcpyAsync(x->f.rho, prob->rho, cb, kind, x->stream)) == hipSuccess &&
          (e = hipMemcpyAsync(x->f.e, prob->e, cb, kind, x->stream)) == hipSuccess &&
          (e = hipMemcpyAsync(x->f.u, prob->u, nb, kind, x->stream)) == hipSuccess &&
          (e = hipMemcpyAsync(x->f.v, prob->v, nb, kind, x->stream)) == hipSuccess &&
          (e = hipMemcpyAsync(x->f.w, prob->w, nb, kind, x->stream)) == hipSuccess) {
        // host sources must not be touched after return: wait for the copies
        if (!prob->user_on_device) e = hipStreamSynchronize(x->stream);
        if (e == hipSuccess)
          e = sale::launch_init_user(m, x->ctl, x->f, t0, prob->step0, x->t_end, x->stream);
      }
    }
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
  HIP_TRY(sale::launch_step_fp64(x->m, x->ctl, x->f, x->stream));
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
  int rc = read_ctl(x, &c);
  if (rc != SALE_OK) return rc;
  if ((rc = status_code(c)) != SALE_OK) return rc;
  int64_t left = max_steps;
  long long last_step = c.step;
  double last_t = c.t;
  int64_t chunk = 4;
  while (left > 0) {
    const int64_t n = std::min(left, chunk);
    for (int64_t s = 0; s < n; s++) {
      hipError_t e = sale::launch_step_fp64(x->m, x->ctl, x->f, x->stream);
      if (e != hipSuccess) return hip_fail(e, "sale_run");
    }
    left -= n;
    if ((rc = read_ctl(x, &c)) != SALE_OK) return rc;
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
  int rc = read_ctl(x, &c);
  if (rc != SALE_OK) return rc;
  if (flags) *flags = (int32_t)c.status;
  return status_code(c);
}

int sale_fields(sale_ctx *x, uint32_t mask, void *const *dst, int dst_on_device, int as_fp64) {
  if (!x || (mask && !dst)) return SALE_EINVAL;
  if (mask & ~((SALE_F_TOTALS << 1) - 1u)) return SALE_EINVAL;
  (void)as_fp64;  // storage is FP64 in this build
  const Mesh &m = x->m;
  const hipMemcpyKind kind = dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  const size_t cb = (size_t)m.ncell * sizeof(double), nb = (size_t)m.nnode * sizeof(double);
  int slot = 0;
  for (uint32_t bit = 1; bit <= SALE_F_TOTALS; bit <<= 1) {
    if (!(mask & bit)) continue;
    void *d = dst[slot++];
    if (!d) return SALE_EINVAL;
    switch (bit) {
      case SALE_F_RHO: HIP_TRY(hipMemcpyAsync(d, x->f.rho, cb, kind, x->stream)); break;
      case SALE_F_E: HIP_TRY(hipMemcpyAsync(d, x->f.e, cb, kind, x->stream)); break;
      case SALE_F_P:
      case SALE_F_Q:
        HIP_TRY(sale::launch_derived_fp64(m, x->f, bit == SALE_F_P ? 0 : 1, x->f.scratch, x->stream));
        HIP_TRY(hipMemcpyAsync(d, x->f.scratch, cb, kind, x->stream));
        // the scratch array is reused by the next derived field: wait
        HIP_TRY(hipStreamSynchronize(x->stream));
        break;
      case SALE_F_U: HIP_TRY(hipMemcpyAsync(d, x->f.u, nb, kind, x->stream)); break;
      case SALE_F_V: HIP_TRY(hipMemcpyAsync(d, x->f.v, nb, kind, x->stream)); break;
      case SALE_F_W: HIP_TRY(hipMemcpyAsync(d, x->f.w, nb, kind, x->stream)); break;
      case SALE_F_STATE: {
        Ctl c;
        int rc = read_ctl(x, &c);
        if (rc != SALE_OK) return rc;
        double *o = (double *)d;
        double amax = 0.0;
        memcpy(&amax, &c.amax_bits, sizeof(amax));
        const double rem = c.t_end - c.t;
        double dtn = amax > 0.0 ? m.cfl * m.h / amax : rem;
        if (dtn > rem) dtn = rem;
        o[0] = c.t;
        o[1] = (double)c.step;
        o[2] = dtn;
        o[3] = (double)c.status;
        break;
      }
      case SALE_F_TOTALS: {
        HIP_TRY(sale::launch_totals_fp64(m, x->ctl, x->f, x->stream));
        Ctl c;
        int rc = read_ctl(x, &c);
        if (rc != SALE_OK) return rc;
        ((double *)d)[0] = c.totals[0];
        ((double *)d)[1] = c.totals[1];
        break;
      }
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

// C ABI of the VLBM MHD library (include/vlbm.h): parameter validation, context
// and buffer ownership, codec set-up, and stream-ordered launches of the kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "vlbm.h"
#include "vlbm_ctx.h"
#include "vlbm_kernels.h"

using namespace vlbm;

namespace {

thread_local std::string g_create_err;

vlbm_status fail(vlbm_ctx* c, vlbm_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c)
    c->err = buf;
  else
    g_create_err = buf;
  return s;
}

vlbm_status hip_fail(vlbm_ctx* c, hipError_t e, const char* what) {
  return fail(c, e == hipErrorOutOfMemory ? VLBM_ERR_OOM : VLBM_ERR_HIP, "%s: %s", what,
              hipGetErrorString(e));
}

#define VLBM_HIP(c, call)                              \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return hip_fail(c, e_, #call); \
  } while (0)

int dim_of(int lattice) { return lattice == VLBM_D3Q7 ? 3 : 2; }
int nvars_of(int model) {
  return model == VLBM_RESISTIVE ? 26
         : (model == VLBM_EULER ? 5 : (model == VLBM_NAVIER_CAUCHY ? 9 : (model == VLBM_RESISTIVE_2D ? 13 : 8)));
}
int esize_of(int storage) {
  switch (storage) {
    case VLBM_F64: return 8;
    case VLBM_F32: return 4;
    default: return 2;
  }
}

// Plane stride in elements: each plane rounded up to 4 KiB plus 4 KiB more, so that
// the same cell of consecutive planes does not fall on the same HBM channel and
// bank when the plane size is a power of two (measured on gfx950: +4 % to +18 %
// sweep bandwidth against unpadded power-of-two planes).
long long plane_stride(long long N, int esize) {
  const long long bytes = (N * esize + 4095) / 4096 * 4096 + 4096;
  return bytes / esize;
}

vlbm_status validate(const vlbm_params* p) {
  if (!p) return fail(nullptr, VLBM_ERR_ARG, "params is NULL");
  if (p->struct_size != sizeof(vlbm_params))
    return fail(nullptr, VLBM_ERR_ARG, "params.struct_size %u != %zu (ABI mismatch)", p->struct_size,
                sizeof(vlbm_params));
  if (p->lattice != VLBM_D2Q5 && p->lattice != VLBM_D3Q7)
    return fail(nullptr, VLBM_ERR_ARG, "unknown lattice %d", p->lattice);
  if (p->nx < 1 || p->ny < 1 || p->nz < 1)
    return fail(nullptr, VLBM_ERR_ARG, "lattice extent %d x %d x %d", p->nx, p->ny, p->nz);
  const long long N = (long long)p->nx * p->ny * p->nz;
  if (N >= (1LL << 31)) return fail(nullptr, VLBM_ERR_ARG, "%lld cells exceed 2^31 - 1", N);
  if (plane_stride(N, esize_of(p->storage)) * esize_of(p->storage) >= (1LL << 32))
    return fail(nullptr, VLBM_ERR_ARG, "one population plane would exceed 4 GiB");
  if (p->model != VLBM_IDEAL && p->model != VLBM_RESISTIVE && p->model != VLBM_EULER &&
      p->model != VLBM_NAVIER_CAUCHY && p->model != VLBM_RESISTIVE_2D)
    return fail(nullptr, VLBM_ERR_ARG, "unknown model %d", p->model);
  if (p->model == VLBM_NAVIER_CAUCHY &&
      (!(p->lame_mu > 0.0) || !(p->rho0 > 0.0) || !(p->lame_lambda + 2.0 * p->lame_mu > 0.0) ||
       !std::isfinite(p->lame_lambda) || !std::isfinite(p->lame_mu) || !std::isfinite(p->rho0)))
    return fail(nullptr, VLBM_ERR_ARG, "Navier-Cauchy needs lame_mu > 0, rho0 > 0, lame_lambda + 2 lame_mu > 0");
  if (p->model == VLBM_RESISTIVE && p->lattice != VLBM_D3Q7)
    return fail(nullptr, VLBM_ERR_ARG, "the resistive model needs D3Q7");
  if (p->model == VLBM_RESISTIVE_2D && p->lattice != VLBM_D2Q5)
    return fail(nullptr, VLBM_ERR_ARG, "the 13-component resistive model needs D2Q5");
  if (p->storage < VLBM_F64 || p->storage > VLBM_BF16DEV)
    return fail(nullptr, VLBM_ERR_ARG, "unknown storage %d", p->storage);
  if (!(p->gamma > 1.0) || !std::isfinite(p->gamma)) return fail(nullptr, VLBM_ERR_ARG, "gamma must be > 1");
  if (!(p->flux_scale > 0.0) || !std::isfinite(p->flux_scale))
    return fail(nullptr, VLBM_ERR_ARG, "flux_scale must be > 0");
  if (!(p->w0 >= 0.0 && p->w0 < 1.0)) return fail(nullptr, VLBM_ERR_ARG, "w0 must be in [0, 1)");
  const int K = nvars_of(p->model);
  for (int k = 0; k < K; ++k)
    if (!(p->tau[k] > 0.5) || !std::isfinite(p->tau[k]))
      return fail(nullptr, VLBM_ERR_ARG, "tau[%d] = %g must be > 0.5", k, p->tau[k]);
  if (p->powell != 0 && p->powell != 1) return fail(nullptr, VLBM_ERR_ARG, "powell must be 0 or 1");
  const bool resistive = p->model == VLBM_RESISTIVE || p->model == VLBM_RESISTIVE_2D;
  if (p->divb_mode != 0 && !(p->divb_mode == 1 && resistive))
    return fail(nullptr, VLBM_ERR_ARG, "divb_mode %d not valid for this model", p->divb_mode);
  if (resistive) {
    if (!(p->tau_M > 0.0) || !(p->tau_H > 0.0) || !(p->dt > 0.0))
      return fail(nullptr, VLBM_ERR_ARG, "resistive model needs dt, tau_M, tau_H > 0");
    if (!(p->mu >= 0.0) || !(p->eta0 >= 0.0)) return fail(nullptr, VLBM_ERR_ARG, "mu, eta0 must be >= 0");
  }
  bool faces = false;
  const int32_t ext[3] = {p->nx, p->ny, p->nz};
  for (int f = 0; f < 6; ++f) {
    if (p->bc[f] < VLBM_BC_PERIODIC || p->bc[f] > VLBM_BC_ZERO_GRAD)
      return fail(nullptr, VLBM_ERR_ARG, "bc[%d] = %d is not a vlbm_bc", f, p->bc[f]);
    if ((p->bc[f] == VLBM_BC_PERIODIC) != (p->bc[f ^ 1] == VLBM_BC_PERIODIC))
      return fail(nullptr, VLBM_ERR_ARG, "faces %d and %d: both periodic or neither", f & ~1, f | 1);
    if (p->bc[f] != VLBM_BC_PERIODIC) {
      faces = true;
      if (ext[f >> 1] < 3) return fail(nullptr, VLBM_ERR_ARG, "non-periodic axis %d needs >= 3 cells", f >> 1);
    }
  }
  if (p->body < 0 || p->body > 2) return fail(nullptr, VLBM_ERR_ARG, "body must be 0, 1 or 2");
  if (p->collision < 0 || p->collision > 3) return fail(nullptr, VLBM_ERR_ARG, "collision must be 0, 1, 2 or 3");
  if (p->source < 0 || p->source > 2) return fail(nullptr, VLBM_ERR_ARG, "source must be 0, 1 or 2");
  if (p->source != 0) {
    if (p->storage != VLBM_F64 && p->storage != VLBM_F32)
      return fail(nullptr, VLBM_ERR_ARG, "the Guo and Chai source operators need FP64 or FP32 storage");
    if (p->model != VLBM_IDEAL && p->model != VLBM_RESISTIVE && p->model != VLBM_RESISTIVE_2D)
      return fail(nullptr, VLBM_ERR_ARG, "the Guo and Chai source operators apply to the models with a source");
    if (faces || p->body) return fail(nullptr, VLBM_ERR_ARG, "the Guo and Chai source operators need a periodic lattice");
  }
  if (p->collision == 3 && (!(p->mrt_tau_e > 0.5) || !(p->mrt_tau_d > 0.5) || !std::isfinite(p->mrt_tau_e) ||
                            !std::isfinite(p->mrt_tau_d)))
    return fail(nullptr, VLBM_ERR_ARG, "MRT needs mrt_tau_e, mrt_tau_d > 0.5");
  if (p->collision == 1 && !(p->trt_magic > 0.0 && std::isfinite(p->trt_magic)))
    return fail(nullptr, VLBM_ERR_ARG, "trt_magic must be > 0");
  if ((faces || p->body) && (p->lattice != VLBM_D3Q7 || p->model != VLBM_IDEAL))
    return fail(nullptr, VLBM_ERR_ARG, "non-periodic faces and the body need the D3Q7 ideal model");
  if (faces || p->body)
    for (int k = 0; k < 8; ++k)
      if (!std::isfinite(p->inflow_Q[k])) return fail(nullptr, VLBM_ERR_ARG, "inflow_Q[%d] not finite", k);
  if (faces && !(p->inflow_Q[0] > 0.0)) return fail(nullptr, VLBM_ERR_ARG, "inflow_Q[0] (density) must be > 0");
  if (p->body) {
    if (!(p->body_R0 > 0.0) || !std::isfinite(p->body_R0)) return fail(nullptr, VLBM_ERR_ARG, "body_R0 must be > 0");
    const double* vals[] = {p->body_c0, p->body_v, p->body_a, &p->body_d[0][0], p->body_b, &p->body_e[0][0],
                            p->body_m};
    const int cnt[] = {3, 3, 4, 12, 4, 12, 3};
    for (int j = 0; j < 7; ++j)
      for (int q = 0; q < cnt[j]; ++q)
        if (!std::isfinite(vals[j][q])) return fail(nullptr, VLBM_ERR_ARG, "body parameters must be finite");
  }
  if (p->block_x != 0 && (p->block_x < 64 || p->block_x > 256 || p->block_x % 64 != 0))
    return fail(nullptr, VLBM_ERR_ARG, "block_x must be 64, 128, 192 or 256");
  if (p->rest_Q)
    for (int k = 0; k < K; ++k)
      if (!std::isfinite(p->rest_Q[k])) return fail(nullptr, VLBM_ERR_ARG, "rest_Q[%d] not finite", k);
  for (int k = 0; k < K; ++k)
    if (!(p->scale[k] >= 0.0) || !std::isfinite(p->scale[k]))
      return fail(nullptr, VLBM_ERR_ARG, "scale[%d] must be >= 0", k);
  return VLBM_OK;
}

// smallest power of two >= v (1 for v == 0)
double pow2_at_least(double v) {
  if (!(v > 0.0)) return 1.0;
  int e;
  const double m = std::frexp(v, &e);  // v = m 2^e, m in [0.5, 1)
  return m == 0.5 ? std::ldexp(1.0, e - 1) : std::ldexp(1.0, e);
}

// FP16/BF16 codec table: f_rest = f^eq(Q_rest), scale w_i sigma_k.
// Cells whose mask can change when the body moves from time t0 to t1 (t0 <= t1):
// the bounding box of both positions, widened by the surface-radius bound and two
// cells (the link bits of the neighbours), clipped to the domain.
void body_box(vlbm_ctx* c, double t0, double t1, int (&box)[6]) {
  const int n[3] = {c->p.nx, c->p.ny, c->p.nz};
  for (int a = 0; a < 3; ++a) {
    const double p0 = c->body.c0[a] + t0 * c->body.v[a], p1 = c->body.c0[a] + t1 * c->body.v[a];
    const double lo = std::floor(std::min(p0, p1) - c->body_rmax) - 2.0;
    const double hi = std::ceil(std::max(p0, p1) + c->body_rmax) + 3.0;
    box[2 * a] = (int)std::max(0.0, std::min((double)n[a], lo));
    box[2 * a + 1] = (int)std::max(0.0, std::min((double)n[a], hi));
  }
}

// Homogenized body at time t: the box of cells within the surface-radius bound plus
// one cell (porosity below 1 possible only there), clipped to the domain.
void hlbm_box(vlbm_ctx* c, double t, int (&box)[6]) {
  const int n[3] = {c->p.nx, c->p.ny, c->p.nz};
  for (int a = 0; a < 3; ++a) {
    const double p0 = c->body.c0[a] + t * c->body.v[a];
    const double lo = std::floor(p0 - c->body_rmax) - 1.0, hi = std::ceil(p0 + c->body_rmax) + 2.0;
    box[2 * a] = (int)std::max(0.0, std::min((double)n[a], lo));
    box[2 * a + 1] = (int)std::max(0.0, std::min((double)n[a], hi));
  }
}

// Mask of the whole lattice at the current step (after init or a restore).
hipError_t body_mask_full(vlbm_ctx* c) {
  Body b = c->body;
  b.t = (double)c->step;
  b.box[0] = b.box[2] = b.box[4] = 0;
  b.box[1] = c->p.nx;
  b.box[3] = c->p.ny;
  b.box[5] = c->p.nz;
  hipError_t e = launch_mask(c->L, c->g, b, 0, 1);
  if (e == hipSuccess) e = launch_mask(c->L, c->g, b, 1, 0);
  return e;
}

void build_codec(vlbm_ctx* c) {
  ++c->gen;
  std::memset(&c->cd, 0, sizeof c->cd);
  if (c->p.storage != VLBM_F16DEV && c->p.storage != VLBM_BF16DEV) return;
  double P[KMAX][3], S[KMAX], dl, Jb[3] = {0, 0, 0};
  if (c->p.model == VLBM_NAVIER_CAUCHY && c->D == 2)
    flux_source<double, 2, 3>(c->rest_Q, Jb, c->ph, P, S, dl);
  else if (c->p.model == VLBM_NAVIER_CAUCHY)
    flux_source<double, 3, 3>(c->rest_Q, Jb, c->ph, P, S, dl);
  else if (c->p.model == VLBM_EULER && c->D == 2)
    flux_source<double, 2, 2>(c->rest_Q, Jb, c->ph, P, S, dl);
  else if (c->p.model == VLBM_EULER)
    flux_source<double, 3, 2>(c->rest_Q, Jb, c->ph, P, S, dl);
  else if (c->p.model == VLBM_RESISTIVE_2D)
    flux_source<double, 2, 4>(c->rest_Q, Jb, c->ph, P, S, dl);
  else if (c->D == 2)
    flux_source<double, 2, 0>(c->rest_Q, Jb, c->ph, P, S, dl);
  else if (c->p.model == VLBM_RESISTIVE)
    flux_source<double, 3, 1>(c->rest_Q, Jb, c->ph, P, S, dl);
  else
    flux_source<double, 3, 0>(c->rest_Q, Jb, c->ph, P, S, dl);
  for (int k = 0; k < c->K; ++k)
    for (int i = 0; i < c->NQ; ++i) {
      const double w = i == 0 ? c->ph.w0 : c->ph.wi;
      double fr;
      if (c->D == 2)
        fr = feq_dir<double, 2>(c->rest_Q[k], P[k], i, c->ph.w0, c->ph.wi);
      else
        fr = feq_dir<double, 3>(c->rest_Q[k], P[k], i, c->ph.w0, c->ph.wi);
      c->cd.rest[k * c->NQ + i] = (float)fr;
      c->cd.sc[k * c->NQ + i] = (float)(w * c->scale[k]);
      c->cd.isc[k * c->NQ + i] = (float)(1.0 / (w * c->scale[k]));
    }
}

}  // namespace

// One step on the context's stream: faces, sweep (with the body, and its move), step + 1.
vlbm_status vlbm_step_one(vlbm_ctx* c) {
  const int par = (int)(c->step & 1);
  Grid g = c->g;
  Body b = c->body;
  b.t = (double)c->step;
  if (c->p.body == 2) {
    hlbm_box(c, b.t, b.box);
    // the box sweep re-sets no face: a box that reaches the x faces (or the cells whose
    // moments a zero-gradient x face takes) leaves them to the face pass this step
    const bool nonempty = b.box[1] > b.box[0] && b.box[3] > b.box[2] && b.box[5] > b.box[4];
    if (g.bc[0] && nonempty && (b.box[0] <= 1 || b.box[1] >= g.nx - 1)) g.xf_pass = 1;
  }
  // bounce-back: every solid cell and every cut link lies in the box of the body's
  // position at this step (the sweep leaves that box to the bounce-back sweep, unless
  // it reaches the x faces)
  if (c->p.body == 1) {
    body_box(c, b.t, b.t, b.box);
    // the body must stay clear of the non-periodic faces: a face node inside the box
    // could be solid or have a cut link, which the faces' re-set does not define
    const int n[3] = {c->p.nx, c->p.ny, c->p.nz};
    for (int a = 0; a < 3; ++a)
      if ((g.bc[2 * a] && b.box[2 * a] <= 0) || (g.bc[2 * a + 1] && b.box[2 * a + 1] >= n[a]))
        return fail(c, VLBM_ERR_STATE,
                    "step %lld: the bounce-back body's box [%d,%d) x [%d,%d) x [%d,%d) reaches a non-periodic face",
                    (long long)c->step, b.box[0], b.box[1], b.box[2], b.box[3], b.box[4], b.box[5]);
  }
  if (c->has_faces) {
    const hipError_t e = launch_faces(c->L, g, c->ph, c->cd, par, c->inflow);
    if (e != hipSuccess) return hip_fail(c, e, "face launch");
  }
  if (!c->p.body) {
    const hipError_t e = launch_sweep(c->L, g, c->ph, c->cd, par, c->inflow);
    if (e != hipSuccess) return hip_fail(c, e, "sweep launch");
    ++c->step;
    return VLBM_OK;
  }
  hipError_t e = launch_sweep_body(c->L, g, c->ph, c->cd, par, b, c->p.body, c->inflow);
  if (e != hipSuccess) return hip_fail(c, e, "sweep launch");
  ++c->step;
  if (c->p.body == 2) return VLBM_OK;  // the homogenized body needs no mask
  // the body moves to its position at the new step; uncovered cells are refilled
  body_box(c, b.t, (double)c->step, b.box);
  b.t = (double)c->step;
  e = launch_mask(c->L, c->g, b, 0, 0);
  if (e == hipSuccess) e = launch_mask(c->L, c->g, b, 1, 0);
  if (e == hipSuccess) e = launch_refill(c->L, c->g, c->ph, c->cd, (int)(c->step & 1), b, c->inflow);
  if (e != hipSuccess) return hip_fail(c, e, "body update");
  return VLBM_OK;
}

extern "C" {

vlbm_status vlbm_params_default(vlbm_params* p) {
  if (!p) return VLBM_ERR_ARG;
  std::memset(p, 0, sizeof *p);
  p->struct_size = sizeof(vlbm_params);
  p->lattice = VLBM_D2Q5;
  p->nx = p->ny = 64;
  p->nz = 1;
  p->model = VLBM_IDEAL;
  p->storage = VLBM_F32;
  p->powell = 1;
  p->gamma = 5.0 / 3.0;
  p->flux_scale = 0.2;
  for (int k = 0; k < VLBM_KMAX; ++k) p->tau[k] = 0.6;
  p->tau_M = p->tau_H = 1.0;
  p->trt_magic = 0.25;
  p->lame_lambda = p->lame_mu = p->rho0 = 1.0;
  p->mrt_tau_e = p->mrt_tau_d = 1.0;
  return VLBM_OK;
}

vlbm_status vlbm_population_bytes(const vlbm_params* p, size_t* bytes) {
  vlbm_status s = validate(p);
  if (s != VLBM_OK) return s;
  if (!bytes) return VLBM_ERR_ARG;
  const int D = dim_of(p->lattice), K = nvars_of(p->model), es = esize_of(p->storage);
  const long long N = (long long)p->nx * p->ny * p->nz;
  *bytes = (size_t)K * (2 * D + 1) * plane_stride(N, es) * es;
  return VLBM_OK;
}

vlbm_status vlbm_create(const vlbm_params* p, vlbm_ctx** out) {
  if (!out) return fail(nullptr, VLBM_ERR_ARG, "out is NULL");
  *out = nullptr;
  vlbm_status s = validate(p);
  if (s != VLBM_OK) return s;
  vlbm_ctx* c = new (std::nothrow) vlbm_ctx();
  if (!c) return fail(nullptr, VLBM_ERR_OOM, "host allocation failed");
  c->p = *p;
  c->p.rest_Q = nullptr;
  c->D = dim_of(p->lattice);
  c->K = nvars_of(p->model);
  c->NQ = 2 * c->D + 1;
  c->esize = esize_of(p->storage);
  c->N = (long long)p->nx * p->ny * p->nz;
  c->stride = plane_stride(c->N, c->esize);
  c->pop_bytes = (size_t)c->K * c->NQ * c->stride * c->esize;
  c->stream = static_cast<hipStream_t>(p->stream);
  static std::atomic<long long> next_uid{1};
  c->uid = next_uid++;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return fail(nullptr, VLBM_ERR_HIP, "hipGetDevice failed");
  }
  if (p->rest_Q) {
    for (int k = 0; k < c->K; ++k) c->rest_Q[k] = p->rest_Q[k];
    c->rest_given = true;
  }
  for (int k = 0; k < c->K; ++k) c->scale[k] = p->scale[k];

  const double w0 = p->w0 > 0.0 ? p->w0 : (c->D == 2 ? 1.0 / 3.0 : 0.25);
  Phys& ph = c->ph;
  ph.s = p->flux_scale;
  ph.gm1 = p->gamma - 1.0;
  ph.inv_cs2 = c->D / (1.0 - w0);
  ph.w0 = w0;
  ph.wi = (1.0 - w0) / (2.0 * c->D);
  for (int k = 0; k < KMAX; ++k) ph.omega[k] = k < c->K ? 1.0 / p->tau[k] : 0.0;
  const int bx = p->model == VLBM_RESISTIVE_2D ? 4 : 5;
  for (int a = 0; a < 3; ++a) ph.inv_tauB[a] = 1.0 / p->tau[bx + a];
  if (p->model == VLBM_RESISTIVE || p->model == VLBM_RESISTIVE_2D) {
    ph.dt_over_tauM = p->dt / p->tau_M;
    ph.dt_over_tauH = p->dt / p->tau_H;
    ph.inv_tauM = 1.0 / p->tau_M;
    ph.inv_tauH = 1.0 / p->tau_H;
    ph.mu = p->mu;
    ph.eta0 = p->eta0;
    ph.inv_jc2 = p->j_c > 0.0 ? 1.0 / (p->j_c * p->j_c) : 0.0;
    ph.divb_scale = p->dt / p->flux_scale;
  }
  ph.lame_lambda = p->lame_lambda;
  ph.lame_mu = p->lame_mu;
  ph.inv_rho0 = p->rho0 > 0.0 ? 1.0 / p->rho0 : 0.0;
  ph.powell = p->powell;
  ph.divb_mode = p->divb_mode;
  ph.collision = p->collision;
  ph.source = p->source;
  for (int k = 0; k < KMAX; ++k) {
    const double tau = k < c->K ? p->tau[k] : 1.0;
    ph.omega_s[k] = p->collision == 1 ? 1.0 / (0.5 + p->trt_magic / (tau - 0.5))
                    : p->collision == 2 ? 1.0
                    : p->collision == 3 ? 1.0 / p->mrt_tau_e
                                        : ph.omega[k];
    ph.omega_d[k] = p->collision == 3 ? 1.0 / p->mrt_tau_d : ph.omega_s[k];
  }

  if (p->pop_buffer) {
    if (p->pop_bytes < c->pop_bytes) {
      delete c;
      return fail(nullptr, VLBM_ERR_ARG, "pop_bytes %zu < required %zu", p->pop_bytes, c->pop_bytes);
    }
    c->f = p->pop_buffer;
    c->owned = false;
  } else {
    hipError_t e = hipMalloc(&c->f, c->pop_bytes);
    if (e != hipSuccess) {
      const size_t want = c->pop_bytes;
      delete c;
      return fail(nullptr, e == hipErrorOutOfMemory ? VLBM_ERR_OOM : VLBM_ERR_HIP,
                  "hipMalloc of %zu population bytes: %s", want, hipGetErrorString(e));
    }
    c->owned = true;
  }
  // defined contents everywhere, including the plane padding (bitwise checkpoints
  // and buffer comparisons between contexts)
  if (hipMemsetAsync(c->f, 0, c->pop_bytes, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess) {
    vlbm_destroy(c);
    return fail(nullptr, VLBM_ERR_HIP, "clearing the population buffer failed");
  }
  c->nblk = (int)std::min<long long>(1024, (c->N + 255) / 256);
  const int NT = c->K + 5;
  hipError_t e = hipMalloc(&c->d_partial, sizeof(double) * (size_t)c->nblk * NT);
  if (e == hipSuccess) e = hipMalloc(&c->d_partial2, sizeof(double) * (size_t)c->nblk);
  if (e == hipSuccess) e = hipMalloc(&c->d_totals, sizeof(double) * (size_t)(NT + 2 * KMAX));
  if (e != hipSuccess) {
    vlbm_destroy(c);
    return fail(nullptr, VLBM_ERR_OOM, "hipMalloc of reduction buffers: %s", hipGetErrorString(e));
  }
  c->g.f = c->f;
  c->g.stride = c->stride;
  // 16-bit storage of the 26-variable model: variable pairs share 32-bit elements
  c->g.pk = (p->model == VLBM_RESISTIVE && (p->storage == VLBM_F16DEV || p->storage == VLBM_BF16DEV)) ? 1 : 0;
  c->g.nx = p->nx;
  c->g.ny = p->ny;
  c->g.nz = p->nz;
  for (int f = 0; f < 6; ++f) {
    c->g.bc[f] = p->bc[f];
    c->has_faces |= p->bc[f] != VLBM_BC_PERIODIC;
  }
  for (int k = 0; k < 8; ++k) c->inflow.q[k] = p->inflow_Q[k];
  if (p->body) {
    Body& b = c->body;
    double delta = 0.0;
    for (int a = 0; a < 3; ++a) {
      b.c0[a] = p->body_c0[a];
      b.v[a] = p->body_v[a];
      b.m[a] = p->body_m[a];
    }
    b.R0 = p->body_R0;
    for (int j = 0; j < 4; ++j) {
      b.a[j] = p->body_a[j];
      b.b[j] = p->body_b[j];
      double dd = 0.0, ee = 0.0;
      for (int a = 0; a < 3; ++a) {
        b.d[j][a] = p->body_d[j][a];
        b.e[j][a] = p->body_e[j][a];
        dd += b.d[j][a] * b.d[j][a];
        ee += b.e[j][a] * b.e[j][a];
      }
      // |d_j . n| <= |d_j|, |(e_j . n)^2 - 1/3| <= |e_j|^2 + 1/3
      delta += std::fabs(b.a[j]) * std::sqrt(dd) + std::fabs(b.b[j]) * (ee + 1.0 / 3.0);
    }
    c->body_rmax = b.R0 * (1.0 + delta);
    b.rmax = c->body_rmax;
    if (p->body == 1) {  // bounce-back keeps a solid/link mask
      if (hipMalloc(&c->d_mask, (size_t)c->N) != hipSuccess ||
          hipMemsetAsync(c->d_mask, 0, (size_t)c->N, c->stream) != hipSuccess) {
        vlbm_destroy(c);
        return fail(nullptr, VLBM_ERR_OOM, "allocation of the body mask failed");
      }
      c->g.mask = c->d_mask;
    }
  }
  if (p->source == 2) {  // Chai's source keeps each cell's previous source
    const size_t bytes = (size_t)c->K * (size_t)c->N * (p->storage == VLBM_F64 ? sizeof(double) : sizeof(float));
    if (hipMalloc(&c->d_sprev, bytes) != hipSuccess) {
      vlbm_destroy(c);
      return fail(nullptr, VLBM_ERR_OOM, "allocation of the previous-source field failed");
    }
    c->g.sprev = c->d_sprev;
  }
  c->L.storage = p->storage;
  c->L.dim = c->D;
  c->L.model = p->model;
  c->L.block_x = p->block_x ? p->block_x : (p->nx >= 256 ? 256 : (p->nx >= 128 ? 128 : 64));
  c->L.stream = c->stream;
  *out = c;
  return VLBM_OK;
}

vlbm_status vlbm_init_fields(vlbm_ctx* c, const void* Q, int q_on_device, int q_is_f32) {
  if (!c) return VLBM_ERR_ARG;
  if (!Q) return fail(c, VLBM_ERR_ARG, "Q is NULL");
  const size_t qbytes = (size_t)c->K * c->N * (q_is_f32 ? 4 : 8);
  const void* dQ = Q;
  void* tmp = nullptr;
  if (!q_on_device) {
    VLBM_HIP(c, hipMalloc(&tmp, qbytes));
    hipError_t e = hipMemcpyAsync(tmp, Q, qbytes, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
      (void)hipFree(tmp);
      return hip_fail(c, e, "copy of Q to the device");
    }
    dQ = tmp;
  }
  vlbm_status st = VLBM_OK;
  hipError_t e = hipSuccess;
  const bool codec = c->p.storage == VLBM_F16DEV || c->p.storage == VLBM_BF16DEV;
  if (codec) {
    double* d_aux = c->d_totals + (c->K + 5);  // KMAX doubles after the totals
    if (!c->rest_given) {
      // Q_rest: domain mean with rho u (and G, H) set to zero
      e = launch_field_reduce(c->L, c->N, c->K, dQ, q_is_f32, 0, nullptr, c->d_partial, c->nblk, d_aux);
      double mean[KMAX];
      if (e == hipSuccess) e = hipMemcpyAsync(mean, d_aux, sizeof(double) * c->K, hipMemcpyDeviceToHost, c->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
      if (e == hipSuccess)
        for (int k = 0; k < c->K; ++k)
          c->rest_Q[k] = c->p.model == VLBM_NAVIER_CAUCHY
                             ? (k <= 2 ? 0.0 : mean[k] / (double)c->N)  // momentum at rest, mean stress
                             : c->p.model == VLBM_RESISTIVE_2D
                                   ? ((k >= 1 && k <= 2) || k >= 6 ? 0.0 : mean[k] / (double)c->N)
                                   : ((k >= 1 && k <= 3) || k >= 8 ? 0.0 : mean[k] / (double)c->N);
    }
    bool need_scale = false;
    for (int k = 0; k < c->K; ++k) need_scale |= !(c->p.scale[k] > 0.0);
    if (e == hipSuccess && need_scale) {
      double* d_rest = d_aux + KMAX;
      double* d_dev = d_aux;
      double dev[KMAX];
      e = hipMemcpyAsync(d_rest, c->rest_Q, sizeof(double) * c->K, hipMemcpyHostToDevice, c->stream);
      if (e == hipSuccess)
        e = launch_field_reduce(c->L, c->N, c->K, dQ, q_is_f32, 1, d_rest, c->d_partial, c->nblk, d_dev);
      if (e == hipSuccess) e = hipMemcpyAsync(dev, d_dev, sizeof(double) * c->K, hipMemcpyDeviceToHost, c->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
      if (e == hipSuccess)
        for (int k = 0; k < c->K; ++k) {
          if (c->p.scale[k] > 0.0) continue;
          // a field uniform at the start (its spread no more than the rounding of its
          // mean) is scaled by its own magnitude: the spread it develops later is
          // unknown, and a scale set by rounding noise would saturate FP16 at once
          const double mag = std::fabs(c->rest_Q[k]);
          c->scale[k] = pow2_at_least(dev[k] > std::ldexp(mag, -20) ? dev[k] : mag);
        }
    }
    if (e == hipSuccess) build_codec(c);
  }
  if (e == hipSuccess) e = launch_init(c->L, c->g, c->ph, c->cd, dQ, q_is_f32);
  if (e == hipSuccess && c->p.body == 1) {
    c->step = 0;
    e = body_mask_full(c);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (tmp) (void)hipFree(tmp);
  if (e != hipSuccess) st = hip_fail(c, e, "init_fields");
  if (st == VLBM_OK) {
    c->step = 0;
    c->initialized = true;
  }
  return st;
}

vlbm_status vlbm_step(vlbm_ctx* c, int32_t n) {
  if (!c) return VLBM_ERR_ARG;
  if (n < 0) return fail(c, VLBM_ERR_ARG, "n = %d < 0", n);
  if (!c->initialized) return fail(c, VLBM_ERR_STATE, "vlbm_step before vlbm_init_fields");
  for (int32_t j = 0; j < n; ++j) {
    const vlbm_status s = vlbm_step_one(c);
    if (s != VLBM_OK) return s;
  }
  return VLBM_OK;
}

vlbm_status vlbm_moments(vlbm_ctx* c, void* Q_out, int out_on_device, int out_is_f32, double* totals) {
  if (!c) return VLBM_ERR_ARG;
  if (!c->initialized) return fail(c, VLBM_ERR_STATE, "vlbm_moments before vlbm_init_fields");
  const size_t nq = (size_t)c->K * c->N;
  double* Qd;
  if (Q_out && out_on_device && !out_is_f32) {
    Qd = static_cast<double*>(Q_out);
  } else {
    if (!c->d_Q) VLBM_HIP(c, hipMalloc(&c->d_Q, sizeof(double) * nq));
    Qd = c->d_Q;
  }
  const int NT = c->K + 5;
  const int par = (int)(c->step & 1);
  VLBM_HIP(c, launch_moments(c->L, c->g, c->ph, c->cd, par, Qd, c->d_partial, c->nblk));
  const bool has_B = c->p.model == VLBM_IDEAL || c->p.model == VLBM_RESISTIVE || c->p.model == VLBM_RESISTIVE_2D;
  if (has_B) VLBM_HIP(c, launch_divc(c->L, c->g, Qd, c->d_partial2, c->nblk));
  VLBM_HIP(c, launch_reduce(c->L, NT, c->d_partial, c->nblk, 1u << (c->K + 2), c->d_totals));
  if (has_B) VLBM_HIP(c, launch_reduce(c->L, 1, c->d_partial2, c->nblk, 0u, c->d_totals + c->K + 3));
  double tot[KMAX + 5];
  VLBM_HIP(c, hipMemcpyAsync(tot, c->d_totals, sizeof(double) * NT, hipMemcpyDeviceToHost, c->stream));
  VLBM_HIP(c, hipStreamSynchronize(c->stream));
  if (!has_B) tot[c->K + 3] = 0.0;  // no field, no divergence
  if (Q_out && Qd != Q_out) {
    if (out_is_f32) {
      if (out_on_device) {
        VLBM_HIP(c, launch_to_f32(c->stream, Qd, static_cast<float*>(Q_out), (long long)nq));
      } else {
        std::vector<double> h(nq);
        VLBM_HIP(c, hipMemcpyAsync(h.data(), Qd, sizeof(double) * nq, hipMemcpyDeviceToHost, c->stream));
        VLBM_HIP(c, hipStreamSynchronize(c->stream));
        float* o = static_cast<float*>(Q_out);
        for (size_t j = 0; j < nq; ++j) o[j] = (float)h[j];
      }
    } else {
      VLBM_HIP(c, hipMemcpyAsync(Q_out, Qd, sizeof(double) * nq,
                                 out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
    }
  }
  VLBM_HIP(c, hipStreamSynchronize(c->stream));
  if (totals) std::memcpy(totals, tot, sizeof(double) * NT);
  bool finite = true;
  for (int j = 0; j < NT; ++j) finite = finite && std::isfinite(tot[j]);
  if (!finite || tot[c->K + 4] > 0.0)
    return fail(c, VLBM_ERR_NONFINITE, "%g unphysical cells (rho <= 0, p < 0 or non-finite)", tot[c->K + 4]);
  return VLBM_OK;
}

}  // extern "C"

namespace {

// Scratch of vlbm_moments_noalloc: the per-workgroup FP64 partials of the moments pass
// (at most 1024 workgroups x (K + 5) values), those of the central div B pass (1024)
// and the reduced totals (K + 5).  One copy per GPU the library runs on, held until
// the process ends.  In host code `scratch` only names the symbol: its device address
// comes from hipGetSymbolAddress, once per device.
constexpr size_t kNoallocBlocks = 1024;
constexpr size_t kScratchDoubles = kNoallocBlocks * (KMAX + 5) + kNoallocBlocks + (KMAX + 5);
static_assert(kScratchDoubles * sizeof(double) == VLBM_MOMENTS_NOALLOC_SCRATCH_BYTES,
              "scratch size and its public statement differ");
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (the device must be current).
hipError_t scratch_address(int dev, double** out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" {

vlbm_status vlbm_moments_noalloc(vlbm_ctx* c, double* Q_out, double* totals) {
  if (!c) return VLBM_ERR_ARG;
  if (!c->initialized) return fail(c, VLBM_ERR_STATE, "vlbm_moments_noalloc before vlbm_init_fields");
  if (!Q_out) return fail(c, VLBM_ERR_ARG, "vlbm_moments_noalloc needs a device FP64 moment field");
  const int NT = c->K + 5;
  const size_t need = (size_t)c->nblk * NT + (size_t)c->nblk + NT;
  if ((size_t)c->nblk > kNoallocBlocks || need > kScratchDoubles)
    return fail(c, VLBM_ERR_ARG, "vlbm_moments_noalloc: %zu scratch doubles needed, %zu available", need,
                kScratchDoubles);
  int dev = -1;
  VLBM_HIP(c, hipGetDevice(&dev));
  if (dev != c->device)
    return fail(c, VLBM_ERR_ARG, "vlbm_moments_noalloc: device %d is current, the context lives on device %d", dev,
                c->device);
  double* base = nullptr;
  VLBM_HIP(c, scratch_address(dev, &base));
  // every partial and total is written before it is read: nothing to clear
  double* partial = base;
  double* partial2 = base + (size_t)c->nblk * NT;
  double* tot_d = partial2 + c->nblk;
  double* Qd = static_cast<double*>(Q_out);
  const int par = (int)(c->step & 1);
  VLBM_HIP(c, launch_moments(c->L, c->g, c->ph, c->cd, par, Qd, partial, c->nblk));
  const bool has_B = c->p.model == VLBM_IDEAL || c->p.model == VLBM_RESISTIVE || c->p.model == VLBM_RESISTIVE_2D;
  if (has_B) VLBM_HIP(c, launch_divc(c->L, c->g, Qd, partial2, c->nblk));
  VLBM_HIP(c, launch_reduce(c->L, NT, partial, c->nblk, 1u << (c->K + 2), tot_d));
  if (has_B) VLBM_HIP(c, launch_reduce(c->L, 1, partial2, c->nblk, 0u, tot_d + c->K + 3));
  double tot[KMAX + 5];
  VLBM_HIP(c, hipMemcpyAsync(tot, tot_d, sizeof(double) * NT, hipMemcpyDeviceToHost, c->stream));
  VLBM_HIP(c, hipStreamSynchronize(c->stream));
  if (!has_B) tot[c->K + 3] = 0.0;
  if (totals) std::memcpy(totals, tot, sizeof(double) * NT);
  bool finite = true;
  for (int j = 0; j < NT; ++j) finite = finite && std::isfinite(tot[j]);
  if (!finite || tot[c->K + 4] > 0.0)
    return fail(c, VLBM_ERR_NONFINITE, "%g unphysical cells (rho <= 0, p < 0 or non-finite)", tot[c->K + 4]);
  return VLBM_OK;
}

vlbm_status vlbm_gather_cells(vlbm_ctx* c, const int64_t* cells, int64_t n, double* out) {
  if (!c) return VLBM_ERR_ARG;
  if (!c->initialized) return fail(c, VLBM_ERR_STATE, "gather before vlbm_init_fields");
  if (n < 0 || (n > 0 && (!cells || !out))) return fail(c, VLBM_ERR_ARG, "bad cell list");
  if (n == 0) return VLBM_OK;
  for (int64_t j = 0; j < n; ++j)
    if (cells[j] < 0 || cells[j] >= c->N) return fail(c, VLBM_ERR_ARG, "cell %lld out of range", (long long)cells[j]);
  long long* d_cells = nullptr;
  double* d_out = nullptr;
  const size_t nout = (size_t)n * c->K * c->NQ;
  VLBM_HIP(c, hipMalloc(&d_cells, sizeof(long long) * n));
  hipError_t e = hipMalloc(&d_out, sizeof(double) * nout);
  if (e == hipSuccess) e = hipMemcpyAsync(d_cells, cells, sizeof(long long) * n, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = launch_gather(c->L, c->g, c->cd, (int)(c->step & 1), c->K, d_cells, n, d_out);
  if (e == hipSuccess) e = hipMemcpyAsync(out, d_out, sizeof(double) * nout, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  (void)hipFree(d_cells);
  if (d_out) (void)hipFree(d_out);
  if (e != hipSuccess) return hip_fail(c, e, "gather_cells");
  return VLBM_OK;
}

vlbm_status vlbm_get_populations(vlbm_ctx* c, void* dst, size_t bytes, int32_t* parity, int64_t* step) {
  if (!c) return VLBM_ERR_ARG;
  if (!dst || bytes != c->pop_bytes) return fail(c, VLBM_ERR_ARG, "need %zu bytes", c->pop_bytes);
  VLBM_HIP(c, hipMemcpyAsync(dst, c->f, bytes, hipMemcpyDeviceToHost, c->stream));
  VLBM_HIP(c, hipStreamSynchronize(c->stream));
  if (parity) *parity = (int32_t)(c->step & 1);
  if (step) *step = c->step;
  return VLBM_OK;
}

vlbm_status vlbm_set_populations(vlbm_ctx* c, const void* src, size_t bytes, int32_t parity, int64_t step) {
  if (!c) return VLBM_ERR_ARG;
  if (!src || bytes != c->pop_bytes) return fail(c, VLBM_ERR_ARG, "need %zu bytes", c->pop_bytes);
  if (step < 0 || (step & 1) != parity) return fail(c, VLBM_ERR_ARG, "parity must equal step & 1");
  if ((c->p.storage == VLBM_F16DEV || c->p.storage == VLBM_BF16DEV) && !c->initialized && !c->rest_given)
    return fail(c, VLBM_ERR_STATE, "FP16/BF16 restore needs rest_Q and scale in the params (or a prior init)");
  if (!c->initialized) build_codec(c);
  VLBM_HIP(c, hipMemcpyAsync(c->f, src, bytes, hipMemcpyHostToDevice, c->stream));
  c->step = step;
  if (c->p.body == 1) VLBM_HIP(c, body_mask_full(c));
  VLBM_HIP(c, hipStreamSynchronize(c->stream));
  c->initialized = true;
  return VLBM_OK;
}

vlbm_status vlbm_get_codec(const vlbm_ctx* c, double* rest_Q, double* scale) {
  if (!c) return VLBM_ERR_ARG;
  for (int k = 0; k < c->K; ++k) {
    if (rest_Q) rest_Q[k] = c->rest_Q[k];
    if (scale) scale[k] = c->scale[k];
  }
  return VLBM_OK;
}

vlbm_status vlbm_get_step(const vlbm_ctx* c, int64_t* step) {
  if (!c || !step) return VLBM_ERR_ARG;
  *step = c->step;
  return VLBM_OK;
}

vlbm_status vlbm_body_loads(vlbm_ctx* c, double* loads) {
  if (!c || !loads) return VLBM_ERR_ARG;
  if (!c->initialized) return fail(c, VLBM_ERR_STATE, "body_loads before init_fields");
  if (c->p.body != 2) return fail(c, VLBM_ERR_ARG, "body_loads needs the homogenized body (body = 2)");
  Body b = c->body;
  b.t = (double)c->step;
  hlbm_box(c, b.t, b.box);
  const int par = (int)(c->step & 1);
  VLBM_HIP(c, launch_body_loads(c->L, c->g, c->ph, c->cd, par, b, c->d_partial, c->nblk));
  VLBM_HIP(c, launch_reduce(c->L, 8, c->d_partial, c->nblk, 0u, c->d_totals));
  VLBM_HIP(c, hipMemcpyAsync(loads, c->d_totals, 8 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  VLBM_HIP(c, hipStreamSynchronize(c->stream));
  return VLBM_OK;
}

void vlbm_destroy(vlbm_ctx* c) {
  if (!c) return;
  if (c->owned && c->f) (void)hipFree(c->f);
  if (c->d_partial) (void)hipFree(c->d_partial);
  if (c->d_partial2) (void)hipFree(c->d_partial2);
  if (c->d_totals) (void)hipFree(c->d_totals);
  if (c->d_Q) (void)hipFree(c->d_Q);
  if (c->d_mask) (void)hipFree(c->d_mask);
  if (c->d_sprev) (void)hipFree(c->d_sprev);
  delete c;
}

const char* vlbm_last_error(const vlbm_ctx* c) { return c ? c->err.c_str() : g_create_err.c_str(); }

vlbm_status vlbm_copy_kernel(void* dst, const void* src, size_t bytes, void* stream) {
  if (!dst || !src || bytes % 16 != 0 || (reinterpret_cast<uintptr_t>(dst) & 15) ||
      (reinterpret_cast<uintptr_t>(src) & 15))
    return fail(nullptr, VLBM_ERR_ARG, "copy needs 16-byte aligned pointers and size");
  const hipError_t e = launch_copy(static_cast<hipStream_t>(stream), dst, src, bytes);
  if (e != hipSuccess) return hip_fail(nullptr, e, "copy kernel");
  return VLBM_OK;
}

}  // extern "C"

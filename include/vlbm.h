/*
 * vlbm.h -- C ABI of the MI355X (gfx950) library of the vectorial lattice
 * Boltzmann method (VLBM) for ideal compressible and resistive MHD.
 *
 * Method (paper: "Lattice Boltzmann Methods for Compressible (Magneto)hydrodynamics"):
 *   every conserved variable Q_k has its own population set f_{k,i} on a D2Q5 or
 *   D3Q7 lattice (Sec. 2.2, VLBM update); each set is relaxed by BGK toward the
 *   linear vector equilibrium f^eq_{k,i} = w_i (Q_k + c_i . Phi_k / c_s^2) whose
 *   first moment carries the physical flux Phi_k (Sec. 2.2, equilibrium and
 *   moments); the Powell source S = -(div B)(0, B, u.B, u) is injected directly
 *   (Sec. 2.3, Powell correction; Sec. 3 intro, BGK with direct injection); the
 *   populations then stream to the neighbour along c_i.  The ideal system carries
 *   Q = (rho, rho u, e_tot, B) (Sec. 2.3, ideal MHD); the resistive system adds the
 *   transported gradient tensors G ~ tau_M grad B and H ~ tau_H grad u
 *   (Sec. 2.2.1 local moments evolution; Sec. 2.3 expanded state and resistive MHD).
 *
 * Conventions
 *   - Every function returns a vlbm_status; errors are negative.  No exception or
 *     abort crosses the ABI.  vlbm_last_error() gives the context's last message.
 *   - Lattice units: dx = dt = 1 on the lattice; the lattice flux is s * Phi with
 *     s = flux_scale = dt/dx in the caller's physical units; sources are multiplied
 *     by the physical dt (Powell: by s times the lattice divergence).
 *   - Moment fields are SoA [K][nz][ny][nx] (x fastest).  Variable order k:
 *     0 rho; 1-3 rho u; 4 e_tot; 5-7 B; resistive only: 8-16 G (G[3a+b] ~ tau_M d_a B_b),
 *     17-25 H (H[3a+b] ~ tau_H d_a u_b); the other models list their own order below.
 *   - Direction order i: 0 rest, then +x, -x, +y, -y (, +z, -z).
 *   - Device pointers are HIP device addresses on the current device; host
 *     pointers are ordinary memory.  The caller owns every buffer it passes,
 *     including a borrowed population buffer; the context owns everything else.
 *   - vlbm_step is asynchronous on the context's stream (no host sync).
 *     vlbm_moments, vlbm_gather_cells, vlbm_get_populations and
 *     vlbm_set_populations synchronise that stream.
 *   - One context must not be used from two host threads at once.
 */
#ifndef VLBM_H
#define VLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vlbm_ctx vlbm_ctx;

typedef enum {
  VLBM_OK = 0,
  VLBM_ERR_ARG = -1,       /* invalid argument or parameter */
  VLBM_ERR_OOM = -2,       /* device allocation failed */
  VLBM_ERR_HIP = -3,       /* a HIP runtime call failed */
  VLBM_ERR_STATE = -4,     /* call out of order (e.g. step before init) */
  VLBM_ERR_NONFINITE = -5  /* moments found rho <= 0, p < 0 or a non-finite value */
} vlbm_status;

typedef enum { VLBM_D2Q5 = 0, VLBM_D3Q7 = 1 } vlbm_lattice;
/* IDEAL: ideal compressible MHD, K = 8 (rho, rho u, E, B; Sec. 2.3).  RESISTIVE:
 * resistive incompressible MHD, K = 26 (+ G, H; D3Q7 only).  EULER: compressible
 * Euler, K = 5 (rho, rho u, E) -- the ideal system without the field, the
 * hydrodynamic limit the scheme covers (Sec. 1, Sec. 2.3): fluxes rho u,
 * rho u u + p I, (E + p) u, p = (gamma - 1)(E - rho |u|^2 / 2), no source. */
/* NAVIER_CAUCHY: linear elastodynamics (the Navier-Cauchy equation, which Sec. 1 and
 * Sec. 2.2 name among the equations the scheme covers), K = 9, in first-order
 * velocity-stress form: momentum density m = rho0 v (k = 0..2) and the symmetric Cauchy
 * stress sigma_xx, yy, zz, xy, xz, yz (k = 3..8); fluxes Phi[m_b][a] = -sigma_ba,
 * Phi[sigma_bc][a] = -(lame_lambda delta_bc v_a + lame_mu (delta_ab v_c + delta_ac v_b)),
 * no source.  P and S waves travel at sqrt((lambda + 2 mu) / rho0) and sqrt(mu / rho0);
 * s times the P speed must stay below c_s^2. */
/* RESISTIVE_2D: the 13-component 2D system of the paper's Brio-Wu test (Sec. 3.1 names
 * it; Sec. 2.3 and 2.2.1 define its parts), D2Q5 only: rho, rho u_x, rho u_y, e_tot,
 * B_x, B_y (k = 0..5), the transported viscous stress T_xx, T_xy, T_yy (k = 6..8) and
 * the transported field gradient G_xx, G_xy, G_yx, G_yy (k = 9..12, G[2a+b] ~ tau_M
 * d_a B_b).  Fluxes of the full system of Sec. 2.3 with tau_v = T / tau_H and grad B =
 * G / tau_M; T is carried with T_ab u_c - mu (delta_ca u_b + delta_cb u_a) and relaxed
 * by -T dt / tau_H, so that it settles at tau_H mu (d_a u_b + d_b u_a); G with
 * G (x) u - I (x) B, relaxed by -G dt / tau_M; eta(j) with j = d_x B_y - d_y B_x.  Takes
 * dt, mu, eta0, j_c, tau_M, tau_H as the 3D resistive model; divb_mode 1: div B =
 * tr G / tau_M. */
typedef enum {
  VLBM_IDEAL = 0,
  VLBM_RESISTIVE = 1,
  VLBM_EULER = 2,
  VLBM_NAVIER_CAUCHY = 3,
  VLBM_RESISTIVE_2D = 4
} vlbm_model;

/* Population storage in HBM.  F64 and F32 store f itself (F64 computes in FP64,
 * F32 in FP32).  F16DEV and BF16DEV store h = (f - f_rest[k][i]) / (w_i sigma_k),
 * rounded to nearest even, and collide in FP32; f_rest = f^eq(Q_rest). */
typedef enum { VLBM_F64 = 0, VLBM_F32 = 1, VLBM_F16DEV = 2, VLBM_BF16DEV = 3 } vlbm_storage;

/* Boundary kind per domain face (x-, x+, y-, y+, z-, z+).  PERIODIC wraps; the
 * equilibrium boundaries of Sec. 2.4 (static boundaries): at the start of every step
 * each node of a non-periodic face takes f := f^eq of its boundary state -- the
 * Dirichlet state inflow_Q if it lies on an INFLOW_EQ face, else (ZERO_GRAD) the
 * moments of the nearest interior cell along the face normals -- and then collides
 * and streams like any node.  Both faces of an axis are periodic or neither is; a
 * non-periodic axis needs at least 3 cells.  Accepted by the D3Q7 ideal model only. */
typedef enum { VLBM_BC_PERIODIC = 0, VLBM_BC_INFLOW_EQ = 1, VLBM_BC_ZERO_GRAD = 2 } vlbm_bc;

#define VLBM_KMAX 26
#define VLBM_PARAMS_VERSION 1

typedef struct {
  uint32_t struct_size;   /* sizeof(vlbm_params); checked for ABI versioning */
  int32_t lattice;        /* vlbm_lattice */
  int32_t nx, ny, nz;     /* lattice extent, each >= 1; for D2Q5, nz > 1 is a batch of nz
                             independent periodic nx x ny lattices (no coupling along z) */
  int32_t model;          /* vlbm_model (resistive requires D3Q7) */
  int32_t storage;        /* vlbm_storage */
  int32_t powell;         /* 1: inject the Powell source (Sec. 2.3), 0: off */
  int32_t divb_mode;      /* div B used by the Powell source: 0 local non-equilibrium
                             estimate -(1/c_s^2) sum_a J[B_a][a] / tau_{B_a};
                             1 (resistive only) trace of G / tau_M */
  double gamma;           /* adiabatic index of the equation of state (Sec. 2.3) */
  double flux_scale;      /* s = dt/dx (> 0) */
  double w0;              /* rest weight; w_i = (1 - w0)/(2 dim), c_s^2 = (1 - w0)/dim;
                             0 selects 1/3 (D2Q5) or 1/4 (D3Q7) */
  double tau[VLBM_KMAX];  /* lattice relaxation time per variable, each > 0.5 */
  double dt;              /* physical time step (resistive sources) */
  double mu, eta0, j_c, tau_M, tau_H; /* resistive: viscosity, resistivity
                             eta = eta0 (1 + (|j|/j_c)^2) (j_c <= 0: constant),
                             relaxation times of G and H (> 0) */
  int32_t bc[6];          /* vlbm_bc per face; all PERIODIC for the periodic configs */
  double inflow_Q[8];     /* Dirichlet state of INFLOW_EQ faces (conserved variables) */
  const double* rest_Q;   /* host, K values: Q_rest of the FP16/BF16 codec; NULL: the
                             domain mean of the Q given to vlbm_init_fields, with
                             rho u (and G, H) set to zero */
  double scale[VLBM_KMAX];/* codec sigma_k (> 0); 0: smallest power of two >=
                             max |Q_k - Q_rest,k| over the initial field, or >= |Q_rest,k|
                             if that spread is within 2^-20 |Q_rest,k| (a field uniform
                             at the start; 1 if both are 0) */
  void* pop_buffer;       /* optional borrowed device buffer for the populations */
  size_t pop_bytes;       /* its size in bytes (>= vlbm_population_bytes()) */
  void* stream;           /* hipStream_t for all work; NULL: the null stream */
  int32_t block_x;        /* threads per block along x for the sweep; 0: default */
  int32_t body;           /* moving rough sphere with a dipole field (D3Q7 ideal):
                             0 none, 1 bounce-back, 2 homogenized (Sec. 2.4) */
  /* Body (an extension; the paper's moving bodies are homogenised, Sec. 2.4): centre
   * c(t) = body_c0 + t body_v (cell units, t in steps); solid where the distance of a
   * cell centre to c(t) is below R0 (1 + sum_j a_j (d_j . n) + sum_j b_j ((e_j . n)^2
   * - 1/3)), n the unit direction; dipole moment body_m at the centre, field
   * (3 (m . r) r - m |r|^2) / |r|^5.  A link from a fluid cell into the body bounces
   * back: rho and e_tot halfway with the moving-wall flux correction
   * -2 w_i c_i . s Phi(u_w) / c_s^2, rho u and B anti-bounce-back -f* + 2 w_i Q_w to
   * rho u_w and the dipole field at the link midpoint, u_w = body_v / flux_scale (the
   * velocity that moves body_v cells per step); cells the body uncovers take f^eq of
   * the mean moments of their neighbours that are fluid before and after the move
   * (inflow_Q if there is none).  Solid cells report zero moments.
   * body = 2, the paper's homogenized LBM (Sec. 2.4): every cell collides toward
   * its homogenized state -- porosity d = clamp(phi + 1/2, 0, 1) from the radial
   * signed distance phi = |r| - R(n) (a transition one cell wide), u^ = d u +
   * (1 - d) u_w and B^ = d B + (1 - d) B_b replace u and B in the equilibrium, the
   * flux and the Powell source, rho and the pressure are kept (e_tot follows);
   * B_b is the dipole field outside R0 and the uniform 2 m / R0^3 inside (a
   * uniformly magnetised sphere).  No mask, no refill; all cells report moments.
   * The body must stay clear of the domain faces (it does not wrap); with body = 1 a
   * step whose box of possibly solid or cut cells (the surface-radius bound plus two
   * cells below and three above) reaches a non-periodic face returns VLBM_ERR_STATE. */
  double body_c0[3], body_v[3], body_R0;
  double body_a[4], body_d[4][3], body_b[4], body_e[4][3];
  double body_m[3];
  /* Collision (Sec. 2.2 admits several): 0 BGK; 1 TRT -- the antisymmetric halves
   * (f_i - f_ibar)/2, which carry the first moment, relax with 1/tau_k and the
   * symmetric halves with 1/tau+_k, (tau+_k - 1/2)(tau_k - 1/2) = trt_magic (> 0);
   * 2 regularized BGK -- f* = f^eq + (1 - 1/tau_k) w_i e_i . J^neq / c_s^2 + w_i S~;
   * 3 MRT -- each set's moments (1, e_a, |e|^2 and the deviatoric second moments
   * e_x^2 - e_y^2 [, e_x^2 + e_y^2 - 2 e_z^2]) relax toward those of f^eq: the first
   * moments with 1/tau_k, the zeroth moment and the trace with 1/mrt_tau_e, the
   * deviatoric ones with 1/mrt_tau_d (each > 0.5); then + w_i S~. */
  int32_t collision;
  double trt_magic;
  /* NAVIER_CAUCHY only: Lame constants (lame_mu > 0, lame_lambda + 2 lame_mu > 0) and
   * density (rho0 > 0) of the elastic medium; defaults 1, 1, 1. */
  double lame_lambda, lame_mu, rho0;
  double mrt_tau_e, mrt_tau_d; /* MRT relaxation times (collision 3); defaults 1 */
  /* Source operator (Sec. 2.2 names direct injection, the Guo and the Chai scheme):
   * 0 direct injection, w_i S~(Q) with Q = sum_i f; 1 Guo -- the state is Q = sum_i f +
   * S~(Q)/2 (two fixed-point iterations from the populations' sum; vlbm_moments
   * reports it, and vlbm_init_fields sets sum_i f = Q - S~(Q)/2), the source entering as
   * (1 - omega_0/2) w_i S~ with omega_0 the zeroth moment's relaxation rate; 2 Chai --
   * the source enters as w_i (S~ + (S~ - S~_prev)/2), S~_prev the cell's source of the
   * previous step, kept by the context (K x N values, started at S~ of the initial
   * state; not part of vlbm_get/set_populations).  1 and 2: FP64/FP32 storage, the ideal,
   * resistive and 13-component models, periodic lattices without a body. */
  int32_t source;
} vlbm_params;

/* Fill *p with defaults (periodic, F32, gamma 5/3, s 0.2, tau 0.6, Powell on, BGK,
 * trt_magic 1/4). */
vlbm_status vlbm_params_default(vlbm_params* p);

/* Bytes of the population buffer for these parameters (K*Q padded planes). */
vlbm_status vlbm_population_bytes(const vlbm_params* p, size_t* bytes);

/* Create a context: validate p, allocate (or adopt) the population buffer and the
 * small FP64 reduction buffers.  No kernel runs.  *out is NULL on error. */
vlbm_status vlbm_create(const vlbm_params* p, vlbm_ctx** out);

/* f := f^eq(Q) in every cell (natural layout), step counter := 0.  Q is SoA
 * [K][nz][ny][nx], FP64 (q_is_f32 = 0) or FP32 (q_is_f32 = 1), on the device
 * (q_on_device = 1) or the host.  Also fixes the FP16/BF16 codec tables (see
 * vlbm_params.rest_Q / scale).  Synchronises. */
vlbm_status vlbm_init_fields(vlbm_ctx* c, const void* Q, int q_on_device, int q_is_f32);

/* Advance n >= 0 steps: per cell, gather the populations (in-place AA pattern),
 * moments, equation of state, fluxes, div B estimate, Powell source, BGK with
 * direct injection, scatter (Sec. 2.2-2.3).  Asynchronous on the context stream. */
vlbm_status vlbm_step(vlbm_ctx* c, int32_t n);

/* Moments of the current populations: Q_out SoA [K][nz][ny][nx] (FP64 or FP32,
 * host or device; may be NULL) and totals (host, may be NULL, K + 5 doubles):
 * [0..K-1] sum_x Q_k; [K] sum_x d; [K+1] sum_x d^2; [K+2] max_x |d|, with d the
 * lattice-unit div B estimate of the Powell source; [K+3] sum_x (central-difference
 * div B of the moment field)^2; [K+4] number of cells with rho <= 0, p < 0 or a
 * non-finite moment.  Accumulated in FP64.  Synchronises.  Returns
 * VLBM_ERR_NONFINITE (after filling the outputs) if [K+4] > 0 or a total is not finite. */
vlbm_status vlbm_moments(vlbm_ctx* c, void* Q_out, int out_on_device, int out_is_f32,
                         double* totals);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): vlbm_moments without any device
 * allocation.  Q_out: device FP64 moment field [K][nz][ny][nx] (required: the central
 * div B pass reads the field from it; the caller owns it).  totals: host, K + 5
 * doubles as in vlbm_moments, or NULL.  The FP64 partial sums live in a static array
 * of VLBM_MOMENTS_NOALLOC_SCRATCH_BYTES bytes per GPU (1024 workgroups x (KMAX + 5)
 * partials, 1024 more, and the totals), which each GPU the library runs on holds
 * until the process ends; every lattice this library accepts fits in it.  All calls
 * on one GPU share that array and overwrite it completely before reading it, so calls
 * that overlap on one GPU (from two host threads or on two streams) race.  The
 * device current at the call must be the one current at vlbm_create.  Synchronises
 * the context's stream.  Errors: VLBM_ERR_ARG (NULL Q_out, another device current,
 * a lattice whose partials would not fit), VLBM_ERR_STATE before vlbm_init_fields,
 * VLBM_ERR_NONFINITE as vlbm_moments. */
#define VLBM_MOMENTS_NOALLOC_SCRATCH_BYTES ((1024 * (VLBM_KMAX + 5) + 1024 + (VLBM_KMAX + 5)) * 8)
vlbm_status vlbm_moments_noalloc(vlbm_ctx* c, double* Q_out, double* totals);

/* Decoded pre-collision populations f_{k,i} at the given cells (host arrays):
 * cells[n] linear indices x + nx (y + ny z); out[n][K][Q] FP64.  Synchronises. */
vlbm_status vlbm_gather_cells(vlbm_ctx* c, const int64_t* cells, int64_t n, double* out);

/* Raw population buffer (storage type, internal padded layout) to / from host
 * memory, with the in-place pattern's parity and the step counter: a bitwise
 * checkpoint.  bytes must equal vlbm_population_bytes(). */
vlbm_status vlbm_get_populations(vlbm_ctx* c, void* dst, size_t bytes, int32_t* parity,
                                 int64_t* step);
vlbm_status vlbm_set_populations(vlbm_ctx* c, const void* src, size_t bytes, int32_t parity,
                                 int64_t step);

/* The codec reference state and scales in use (host arrays of K doubles). */
vlbm_status vlbm_get_codec(const vlbm_ctx* c, double* rest_Q, double* scale);

/* Number of steps taken since vlbm_init_fields. */
vlbm_status vlbm_get_step(const vlbm_ctx* c, int64_t* step);

/* Loads on the homogenized body (body = 2) for the context's next step -- the per-step
 * surface integrals of the paper's moving-body showcase (Sec. 5: magnetic flux, force,
 * torque, electromagnetic work) for the homogenization of Sec. 2.4.  The collision
 * moves each cell's conserved variables by omega_k (Q^_k - Q_k) toward its
 * homogenized state; the body receives the opposite.  loads (host, 8 doubles):
 * [0..2] force = -sum omega_m rho (u^ - u) (momentum per step, cell volume 1, flux
 * units); [3..5] torque = -sum (x - c(t)) x omega_m rho (u^ - u) about the body's
 * centre c(t) = body_c0 + t body_v; [6] energy moved to the body per step, -sum
 * omega_E (e^ - e_tot); [7] magnetic flux through the surface, 1/2 sum |B . r/|r||
 * over the one-cell porosity ramp (the surface measure |grad d| dV).  omega_k =
 * 1/tau_k (BGK), the symmetric rate (TRT), 1 (RLB).  Periodic, Powell off: the
 * fluid's momentum and energy totals change in the step by exactly -force, -energy.
 * Synchronises the stream.  VLBM_ERR_ARG without the homogenized body. */
vlbm_status vlbm_body_loads(vlbm_ctx* c, double* loads);

/* Free everything the context owns (never a borrowed buffer).  NULL-safe. */
void vlbm_destroy(vlbm_ctx* c);

/* Last error message of the context ("" if none); NULL context: last create error. */
const char* vlbm_last_error(const vlbm_ctx* c);

/* Plain device-to-device copy of `bytes` bytes (multiple of 16, 16-byte aligned
 * device pointers) with the library's streaming copy kernel, on `stream`: the
 * measured-bandwidth denominator of the roofline.  Asynchronous. */
vlbm_status vlbm_copy_kernel(void* dst, const void* src, size_t bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* VLBM_H */

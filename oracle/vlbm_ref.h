/*
 * Plain FP64 CPU oracle of the vectorial lattice Boltzmann method (VLBM) for
 * ideal compressible and resistive MHD.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  It shares no code,
 * header, table or constant with the GPU library; it is written straight from
 * the paper, in the paper's order, with plain loops and two-lattice push
 * streaming (not the in-place scheme the GPU uses).
 *
 * Paper: "Lattice Boltzmann Methods for Compressible (Magneto)hydrodynamics",
 * Sec. 2.2 (VLBM update, linear vector equilibrium, moments), Sec. 2.2.1
 * (local moments evolution), Sec. 2.3 (MHD state, fluxes, equation of state,
 * Powell source), Sec. 3 intro (BGK collision + direct source injection).
 *
 * Layout: moments Q[k][cell]; populations f[k][i][cell]; cell = x + nx*(y + ny*z).
 * Directions: i = 0 rest, i = 2a+1 is +e_a, i = 2a+2 is -e_a (a = 0..dim-1).
 */
#ifndef VLBM_REF_H
#define VLBM_REF_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VREF_KMAX 26

typedef struct {
  int32_t dim;        /* 2: D2Q5, 3: D3Q7 */
  int32_t nx, ny, nz; /* nz must be 1 when dim == 2 */
  int32_t model;      /* 0: ideal MHD (K = 8); 1: resistive MHD with G, H (K = 26);
                         2: compressible Euler (K = 5); 3: linear elastodynamics
                         (Navier-Cauchy) in velocity-stress form (K = 9); 4: the
                         13-component 2D resistive system (rho, rho u_x, rho u_y,
                         e_tot, B_x, B_y, transported stress xx xy yy relaxed with
                         tau_H, G xx xy yx yy relaxed with tau_M; D2Q5 only) */
  int32_t powell;     /* 1: Powell source injected, 0: off */
  int32_t divb_mode;  /* 0: local non-equilibrium estimate of div B; 1: trace of G / tau_M */
  int32_t reserved;
  double gamma;       /* adiabatic index */
  double s;           /* flux scale dt/dx: lattice flux = s * physical flux */
  double w0;          /* rest weight; w_i = (1-w0)/(2 dim), c_s^2 = (1-w0)/dim */
  double tau[VREF_KMAX]; /* lattice relaxation time per variable (> 0.5) */
  double dt;          /* physical time step (resistive model sources) */
  double mu, eta0, j_c, tau_M, tau_H; /* resistive model; j_c <= 0: constant eta */
  /* boundaries (vref_run_bc only): per face x-, x+, y-, y+, z-, z+:
   * 0 periodic, 1 inflow (equilibrium of inflow_Q), 2 zero gradient (equilibrium of
   * the moments of the nearest interior cell) */
  int32_t bc[6];
  int32_t body;       /* moving rough sphere with a dipole field: 0 none, 1 bounce-back,
                         2 homogenized (porosity blending of Sec. 2.4) */
  double inflow_Q[8];
  /* body: centre c(t) = c0 + t v (cell units, time in steps); surface radius along
   * the unit direction n: R0 (1 + sum_j a_j (d_j . n) + sum_j b_j ((e_j . n)^2 - 1/3));
   * dipole moment m at the centre: B(r) = (3 (m . r) r - m |r|^2) / |r|^5 */
  double body_c0[3], body_v[3], body_R0;
  double body_a[4], body_d[4][3], body_b[4], body_e[4][3];
  double body_m[3];
  /* collision (Sec. 2.2 admits several): 0 BGK, 1 TRT with magic parameter
   * trt_magic, 2 regularized BGK, 3 MRT (first moments at 1/tau_k, the zeroth moment
   * and the trace of the second moments at 1/mrt_tau_e, their deviatoric part at
   * 1/mrt_tau_d) */
  int32_t collision;
  int32_t reserved2;
  double trt_magic;
  /* model 3: Lame constants and density of the elastic medium */
  double lame_lambda, lame_mu, rho0;
  double mrt_tau_e, mrt_tau_d;
  /* source operator (Sec. 2.2 names direct injection, Guo's and Chai's): 0 direct
   * injection, w_i S~(Q), Q = sum_i f; 1 Guo -- the state is Q = sum_i f + S~(Q)/2
   * (solved by two fixed-point iterations from sum_i f) and the source enters as
   * (1 - omega_0/2) w_i S~(Q), omega_0 the relaxation rate of the zeroth moment;
   * 2 Chai -- Q = sum_i f and the source enters as w_i (S~ + (S~ - S~_prev)/2), S~_prev
   * the cell's source of the previous step (the backward difference of dt^2/2 d_t S) */
  int32_t source;
  int32_t reserved3;
} vref_params;

/* number of variables K and of directions Q */
int vref_nvars(const vref_params* p);
int vref_ndirs(const vref_params* p);

/* Physical flux Phi[k][beta] (beta = 0..2) and lattice source S~[k] (Powell and,
 * for the resistive model, the relaxation of G and H) of one cell.
 * J[k][a] = first moment sum_i e_ia f_{k,i} of the cell's populations (used by the
 * local div B estimate).  Writes the lattice div B estimate to *dlat.  Returns 0, or
 * 1 if the cell is unphysical (rho <= 0, p < 0 or a non-finite value). */
int vref_flux_source(const vref_params* p, const double* Q, const double* J,
                     double* Phi /*[K][3]*/, double* S /*[K]*/, double* dlat);

/* f^eq_{k,i} = w_i (Q_k + s e_i . Phi_k / c_s^2) at one cell. */
void vref_equilibrium(const vref_params* p, const double* Q, double* feq /*[K][Q]*/);

/* One collision with direct source injection at one cell; BGK:
 * fstar_{k,i} = f_{k,i} - (f_{k,i} - f^eq_{k,i}) / tau_k + w_i S~_k (TRT and RLB as
 * selected by p->collision). */
int vref_collide(const vref_params* p, const double* f /*[K][Q]*/, double* fstar, double* dlat);

/* vref_collide on n independent cells; f and fstar are [n][K][Q]. */
int vref_collide_many(const vref_params* p, long n, const double* f, double* fstar);
/* Collision of n cells at coordinates xyz [n][3] (time t): with the homogenized body
 * (p->body == 2) each cell collides toward its homogenized state, else as above. */
int vref_collide_at(const vref_params* p, long n, const double* f, const int* xyz, double t, double* fstar);

/* f := f^eq(Q) everywhere. Q is [K][N], f is [K][Q][N]. */
int vref_init(const vref_params* p, const double* Q, double* f);

/* nsteps collide + push-stream steps (periodic). work has the size of f.  Not for
 * the Chai source (source 2), which needs vref_run_src. */
int vref_run(const vref_params* p, double* f, double* work, int nsteps);
/* As vref_run, with the previous-step source sprev [K][N] of the Chai scheme (read
 * and updated; may be NULL for the other source operators). */
int vref_run_src(const vref_params* p, double* f, double* work, double* sprev, int nsteps);
/* The source S~ [K][N] of the state in f (Guo: of Q = sum f + S~/2): the Chai scheme's
 * sprev at the start of a run. */
int vref_source_field(const vref_params* p, const double* f, double* S_out);

/* Moments of f: Q_out [K][N] (may be NULL), dlat [N] (may be NULL), totals (may be
 * NULL): [0..K-1] sum_x Q_k, [K] sum d, [K+1] sum d^2, [K+2] max |d|,
 * [K+3] sum_x (central div B)^2, [K+4] number of unphysical cells. */
int vref_moments(const vref_params* p, const double* f, double* Q_out, double* dlat,
                 double* totals);

/* Sec. 2.4 static boundaries and a moving body: nsteps steps with the face kinds
 * of p->bc and, if p->body, the moving rough sphere.  t0 = time (steps) of the
 * state in f.  Face nodes emit f^eq of their boundary state instead of colliding;
 * body 1: links from a fluid cell into the body bounce back (rho, e_tot: halfway
 * bounce-back with the moving-wall flux correction; rho u, B: anti-bounce-back to
 * the wall values rho u_w and the dipole field); cells the body uncovers are
 * refilled with f^eq of the mean moments of their fluid neighbours.
 * body 2: every cell collides toward its homogenized state (porosity blending of
 * u and B with the body's velocity and field).  work has the size of f. */
int vref_run_bc(const vref_params* p, double* f, double* work, int nsteps, int t0);

/* 1 if cell (x, y, z) is inside the body at time t (steps). */
int vref_solid(const vref_params* p, int x, int y, int z, double t);

/* Lattice porosity d in [0, 1] of the homogenized body at cell (x, y, z), time t. */
double vref_porosity(const vref_params* p, int x, int y, int z, double t);

int vref_num_threads(void);
/* Set the number of OpenMP threads the oracle uses (n >= 1). */
void vref_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif

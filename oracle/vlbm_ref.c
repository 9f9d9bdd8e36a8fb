/*
 * Plain FP64 CPU oracle of the VLBM for MHD.  TEST INFRASTRUCTURE ONLY: it is
 * loaded by the tests, the smoke check and the CPU-baseline leg of the
 * benchmark, never by the product path.  See vlbm_ref.h for layout and ABI.
 *
 * Every function follows the paper ("Lattice Boltzmann Methods for Compressible
 * (Magneto)hydrodynamics") in its own order and notation; readings of points the
 * paper leaves open are marked READING and are the ones listed in the design notes.
 */
#include "vlbm_ref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int vref_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void vref_set_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int vref_nvars(const vref_params* p) {
  return p->model == 1 ? 26 : (p->model == 2 ? 5 : (p->model == 3 ? 9 : (p->model == 4 ? 13 : 8)));
}
/* index of B_x in the state vector: 4 in the 13-component 2D system, else 5 */
static int bx_index(const vref_params* p) { return p->model == 4 ? 4 : 5; }
int vref_ndirs(const vref_params* p) { return 2 * p->dim + 1; }

/* Lattice (Sec. 2.2; the paper's lattice table is not printed).
 * READING: D2Q5/D3Q7 with rest weight w0 and w_i = (1-w0)/(2 dim) for the 2 dim
 * moving directions, so that sum_i w_i = 1 and sum_i w_i e_i e_i = c_s^2 I with
 * c_s^2 = (1-w0)/dim. */
static double weight(const vref_params* p, int i) {
  return i == 0 ? p->w0 : (1.0 - p->w0) / (2.0 * p->dim);
}
static double cs2(const vref_params* p) { return (1.0 - p->w0) / p->dim; }
/* component a of direction i */
static int edir(int i, int a) {
  if (i == 0) return 0;
  int axis = (i - 1) / 2;
  if (axis != a) return 0;
  return (i % 2 == 1) ? 1 : -1;
}

/* Sec. 2.3: state Q = (rho, rho u, e_tot, B [, G, H]) and its physical flux.
 * Ideal part: Phi_rho = rho u; Phi_m = rho u (x) u + p_tot I - B (x) B;
 * Phi_E = (e_tot + p_tot) u - B (u.B); Phi_B = u (x) B - B (x) u, written per
 * component as Phi[B_a][b] = u_b B_a - B_b u_a so that d_t B_a + d_b Phi[B_a][b]
 * is the induction equation.  Equation of state: p = (gamma-1)(e_tot - rho|u|^2/2
 * - |B|^2/2), p_tot = p + |B|^2/2.
 * Resistive part (Sec. 2.2.1 and the expanded state of Sec. 2.3): G_ab ~ tau_M d_a B_b
 * and H_ab ~ tau_H d_a u_b are transported with fluxes G (x) u - I (x) B and
 * H (x) u - I (x) u and relaxed by -G/tau_M, -H/tau_H.
 * READING (garbled stress): viscous stress tau_v = mu (grad u + grad u^T), whose
 * divergence is mu Lap u for a solenoidal flow; heat flux q = 0;
 * eta(j) = eta0 (1 + (|j|/j_c)^2) (constant eta0 when j_c <= 0);
 * j = curl B; the induction flux gains -eta d_b B_a. */
/* Compressible Euler (model 2): the conservation laws of mass, momentum and energy
 * without a field -- the hydrodynamic limit of the MHD system (Sec. 1, Sec. 2.3):
 * Phi = (rho u, rho u u + p I, (E + p) u), p = (gamma - 1)(E - rho |u|^2 / 2), S = 0. */
static int euler_flux(const vref_params* p, const double* Q, double* Phi, double* S, double* dlat) {
  const double rho = Q[0], E = Q[4];
  double u[3], uu = 0.0;
  for (int a = 0; a < 3; ++a) {
    u[a] = Q[1 + a] / rho;
    uu += u[a] * u[a];
  }
  const double pres = (p->gamma - 1.0) * (E - 0.5 * rho * uu);
  for (int b = 0; b < 3; ++b) {
    Phi[3 * 0 + b] = Q[1 + b];
    for (int a = 0; a < 3; ++a) Phi[3 * (1 + a) + b] = Q[1 + a] * u[b] + (a == b ? pres : 0.0);
    Phi[3 * 4 + b] = (E + pres) * u[b];
  }
  for (int k = 0; k < 5; ++k) S[k] = 0.0;
  *dlat = 0.0;
  int bad = !(rho > 0.0) || !(pres >= 0.0);
  for (int k = 0; k < 5; ++k)
    if (!isfinite(Q[k])) bad = 1;
  return bad;
}

/* Linear Navier-Cauchy (model 3), which Sec. 1 and Sec. 2.2 name among the equations
 * the (Q, Phi, S) form covers, written as a first-order system in the momentum
 * density m = rho0 v and the Cauchy stress sigma (symmetric; stored xx, yy, zz, xy,
 * xz, yz):
 *   d_t m_b     = d_a sigma_ba
 *   d_t sigma_bc = lambda delta_bc d_a v_a + mu (d_b v_c + d_c v_b)
 * so Phi[m_b][a] = -sigma_ba and Phi[sigma_bc][a] = -(lambda delta_bc v_a +
 * mu (delta_ab v_c + delta_ac v_b)); no source.  The displacement form
 * rho0 d_t^2 u = mu Lap u + (lambda + mu) grad div u follows for v = d_t u. */
static const int kSigIdx[3][3] = {{3, 6, 7}, {6, 4, 8}, {7, 8, 5}};

static int elastic_flux(const vref_params* p, const double* Q, double* Phi, double* S, double* dlat) {
  const double lam = p->lame_lambda, mu = p->lame_mu;
  double v[3];
  for (int a = 0; a < 3; ++a) v[a] = Q[a] / p->rho0;
  for (int a = 0; a < 3; ++a) {
    for (int b = 0; b < 3; ++b) Phi[3 * b + a] = -Q[kSigIdx[b][a]];
    for (int b = 0; b < 3; ++b)
      for (int c = b; c < 3; ++c)
        Phi[3 * kSigIdx[b][c] + a] = -((b == c ? lam * v[a] : 0.0) + mu * ((a == b ? v[c] : 0.0) + (a == c ? v[b] : 0.0)));
  }
  for (int k = 0; k < 9; ++k) S[k] = 0.0;
  *dlat = 0.0;
  int bad = 0;
  for (int k = 0; k < 9; ++k)
    if (!isfinite(Q[k])) bad = 1;
  return bad;
}

/* The 13-component 2D system of the Brio-Wu test (model 4; Sec. 3.1 names its 13
 * components, Sec. 2.3 defines them): the in-plane state rho, rho u_x, rho u_y, e_tot,
 * B_x, B_y, the transported viscous stress tau (symmetric: xx, xy, yy) and the
 * transported field gradient G (G[2a+b] ~ tau_M d_a B_b: xx, xy, yx, yy), on D2Q5.
 * Fluxes as in the full system of Sec. 2.3 (viscous stress tau_v in the momentum and
 * energy fluxes, -eta grad B in the induction flux, eta j x B in the energy flux,
 * with j = d_x B_y - d_y B_x out of the plane and grad B = G / tau_M); G is carried
 * with G (x) u - I (x) B and relaxed by -G / tau_M (Sec. 2.2.1).
 * READING ("a similar expansion logic is applied to the viscous stress tensor"): the
 * transported stress T_ab is carried with T_ab u_c - mu (delta_ca u_b + delta_cb u_a)
 * and relaxed by -T / tau_H, so that it settles at tau_H mu (d_a u_b + d_b u_a), the
 * stress the 3D system builds from its transported velocity gradient H, and
 * tau_v = T / tau_H.  Powell's source takes div B = tr G / tau_M (divb_mode 1) or the
 * local estimate from the first moments of the B sets (divb_mode 0). */
static int resistive2d_flux(const vref_params* p, const double* Q, const double* J, double* Phi, double* S,
                            double* dlat) {
  const double rho = Q[0], E = Q[3];
  const double u[2] = {Q[1] / rho, Q[2] / rho};
  const double B[2] = {Q[4], Q[5]};
  const double* T = Q + 6; /* xx, xy, yy */
  const double* G = Q + 9; /* xx, xy, yx, yy */
  const double uu = u[0] * u[0] + u[1] * u[1], BB = B[0] * B[0] + B[1] * B[1];
  const double uB = u[0] * B[0] + u[1] * B[1];
  const double pres = (p->gamma - 1.0) * (E - 0.5 * rho * uu - 0.5 * BB);
  const double ptot = 0.5 * BB + pres; /* total pressure */
  double dB[2][2], tv[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) dB[a][b] = G[2 * a + b] / p->tau_M;
  const int tidx[2][2] = {{0, 1}, {1, 2}};
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) tv[a][b] = T[tidx[a][b]] / p->tau_H;
  const double j = dB[0][1] - dB[1][0];
  double eta = p->eta0;
  if (p->j_c > 0.0) eta = p->eta0 * (1.0 + j * j / (p->j_c * p->j_c));
  const double jxB[2] = {-j * B[1], j * B[0]};
  for (int k = 0; k < 13; ++k) {
    S[k] = 0.0;
    for (int c = 0; c < 3; ++c) Phi[3 * k + c] = 0.0;
  }
  for (int c = 0; c < 2; ++c) {
    Phi[3 * 0 + c] = Q[1 + c];
    double utv = 0.0;
    for (int a = 0; a < 2; ++a) {
      Phi[3 * (1 + a) + c] = Q[1 + a] * u[c] + (a == c ? ptot : 0.0) - B[a] * B[c] - tv[a][c];
      utv += u[a] * tv[a][c];
      Phi[3 * (4 + a) + c] = u[c] * B[a] - B[c] * u[a] - eta * dB[c][a];
    }
    Phi[3 * 3 + c] = (E + ptot) * u[c] - B[c] * uB - utv + eta * jxB[c];
    for (int a = 0; a < 2; ++a)
      for (int b = a; b < 2; ++b)
        Phi[3 * (6 + tidx[a][b]) + c] =
            T[tidx[a][b]] * u[c] - p->mu * ((c == a ? u[b] : 0.0) + (c == b ? u[a] : 0.0));
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) Phi[3 * (9 + 2 * a + b) + c] = G[2 * a + b] * u[c] - (a == c ? B[b] : 0.0);
  }
  for (int q = 0; q < 3; ++q) S[6 + q] = -T[q] * p->dt / p->tau_H;
  for (int q = 0; q < 4; ++q) S[9 + q] = -G[q] * p->dt / p->tau_M;
  double divB_lat;
  if (p->divb_mode == 1) {
    divB_lat = (dB[0][0] + dB[1][1]) * (p->dt / p->s);
  } else {
    divB_lat = 0.0;
    for (int a = 0; a < 2; ++a) divB_lat -= J[3 * (4 + a) + a] / p->tau[4 + a];
    divB_lat /= cs2(p);
  }
  *dlat = divB_lat;
  if (p->powell) {
    const double cp = -p->s * divB_lat;
    for (int a = 0; a < 2; ++a) {
      S[1 + a] += cp * B[a];
      S[4 + a] += cp * u[a];
    }
    S[3] += cp * uB;
  }
  int bad = !(rho > 0.0) || !(pres >= 0.0);
  for (int k = 0; k < 13; ++k)
    if (!isfinite(Q[k])) bad = 1;
  return bad;
}

int vref_flux_source(const vref_params* p, const double* Q, const double* J,
                     double* Phi, double* S, double* dlat) {
  if (p->model == 2) return euler_flux(p, Q, Phi, S, dlat);
  if (p->model == 3) return elastic_flux(p, Q, Phi, S, dlat);
  if (p->model == 4) return resistive2d_flux(p, Q, J, Phi, S, dlat);
  const int K = vref_nvars(p);
  const int d = p->dim;
  const double g = p->gamma;
  const double rho = Q[0];
  const double m[3] = {Q[1], Q[2], Q[3]};
  const double E = Q[4];
  const double B[3] = {Q[5], Q[6], Q[7]};
  double u[3];
  for (int a = 0; a < 3; ++a) u[a] = m[a] / rho;
  double uu = 0.0, BB = 0.0, uB = 0.0;
  for (int a = 0; a < 3; ++a) {
    uu += u[a] * u[a];
    BB += B[a] * B[a];
    uB += u[a] * B[a];
  }
  const double pres = (g - 1.0) * (E - 0.5 * rho * uu - 0.5 * BB);
  const double ptot = pres + 0.5 * BB;

  for (int k = 0; k < K; ++k) {
    S[k] = 0.0;
    for (int b = 0; b < 3; ++b) Phi[3 * k + b] = 0.0;
  }
  for (int b = 0; b < 3; ++b) {
    Phi[3 * 0 + b] = m[b];
    for (int a = 0; a < 3; ++a)
      Phi[3 * (1 + a) + b] = m[a] * u[b] + (a == b ? ptot : 0.0) - B[a] * B[b];
    Phi[3 * 4 + b] = (E + ptot) * u[b] - B[b] * uB;
    for (int a = 0; a < 3; ++a) Phi[3 * (5 + a) + b] = u[b] * B[a] - B[b] * u[a];
  }

  double divB_lat; /* lattice-unit divergence of B used by the Powell source */
  if (p->model == 1) {
    const double* G = Q + 8;  /* G[3a+b] ~ tau_M d_a B_b */
    const double* H = Q + 17; /* H[3a+b] ~ tau_H d_a u_b */
    double dB[3][3], du[3][3];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        dB[a][b] = G[3 * a + b] / p->tau_M;
        du[a][b] = H[3 * a + b] / p->tau_H;
      }
    const double jc[3] = {dB[1][2] - dB[2][1], dB[2][0] - dB[0][2], dB[0][1] - dB[1][0]};
    double eta = p->eta0;
    if (p->j_c > 0.0) {
      const double jj = jc[0] * jc[0] + jc[1] * jc[1] + jc[2] * jc[2];
      eta = p->eta0 * (1.0 + jj / (p->j_c * p->j_c));
    }
    const double jxB[3] = {jc[1] * B[2] - jc[2] * B[1], jc[2] * B[0] - jc[0] * B[2],
                           jc[0] * B[1] - jc[1] * B[0]};
    double tv[3][3];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) tv[a][b] = p->mu * (du[a][b] + du[b][a]);
    for (int b = 0; b < 3; ++b) {
      for (int a = 0; a < 3; ++a) Phi[3 * (1 + a) + b] -= tv[a][b];
      double utv = 0.0;
      for (int a = 0; a < 3; ++a) utv += u[a] * tv[a][b];
      Phi[3 * 4 + b] += -utv + eta * jxB[b];
      for (int a = 0; a < 3; ++a) Phi[3 * (5 + a) + b] -= eta * dB[b][a];
    }
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b)
        for (int c = 0; c < 3; ++c) {
          Phi[3 * (8 + 3 * a + b) + c] = G[3 * a + b] * u[c] - (c == a ? B[b] : 0.0);
          Phi[3 * (17 + 3 * a + b) + c] = H[3 * a + b] * u[c] - (c == a ? u[b] : 0.0);
        }
    /* relaxation sources of the transported gradients, times the time step */
    for (int q = 0; q < 9; ++q) {
      S[8 + q] = -G[q] * p->dt / p->tau_M;
      S[17 + q] = -H[q] * p->dt / p->tau_H;
    }
    if (p->divb_mode == 1) {
      double tr = 0.0;
      for (int a = 0; a < d; ++a) tr += dB[a][a];
      divB_lat = tr * (p->dt / p->s); /* physical divergence times dx */
    } else {
      divB_lat = 0.0;
      for (int a = 0; a < d; ++a) divB_lat += J[3 * (5 + a) + a] / p->tau[5 + a];
      divB_lat *= -1.0 / cs2(p);
    }
  } else {
    /* READING (div B for the 8-variable system): local non-equilibrium estimate.
     * The first moment of the B_a set deviates from its equilibrium value s Phi[B_a]
     * by about -tau c_s^2 grad B_a, and Phi[B_a][a] = 0, so
     * div B ~ -(1/c_s^2) sum_a J[B_a][a] / tau_{B_a}. */
    divB_lat = 0.0;
    for (int a = 0; a < d; ++a) divB_lat += J[3 * (5 + a) + a] / p->tau[5 + a];
    divB_lat *= -1.0 / cs2(p);
  }
  *dlat = divB_lat;

  /* Powell source S = -(div B) (0, B, u.B, u) (Sec. 2.3); on the lattice the
   * physical divergence is divB_lat / dx and the source is multiplied by dt. */
  if (p->powell) {
    const double c = -p->s * divB_lat;
    for (int a = 0; a < 3; ++a) {
      S[1 + a] += c * B[a];
      S[5 + a] += c * u[a];
    }
    S[4] += c * uB;
  }
  int bad = !(rho > 0.0) || !(pres >= 0.0);
  for (int k = 0; k < K; ++k)
    if (!isfinite(Q[k])) bad = 1;
  return bad;
}

/* Sec. 2.2: linear vector equilibrium f^eq_{k,i} = w_i (Q_k + c_i . Phi_k / c_s^2),
 * with the lattice flux s Phi. */
static void equilibrium_from_flux(const vref_params* p, const double* Q, const double* Phi,
                                  double* feq) {
  const int K = vref_nvars(p), NQ = vref_ndirs(p), d = p->dim;
  const double c2 = cs2(p);
  for (int k = 0; k < K; ++k)
    for (int i = 0; i < NQ; ++i) {
      double ephi = 0.0;
      for (int a = 0; a < d; ++a) ephi += edir(i, a) * p->s * Phi[3 * k + a];
      feq[k * NQ + i] = weight(p, i) * (Q[k] + ephi / c2);
    }
}

void vref_equilibrium(const vref_params* p, const double* Q, double* feq) {
  double Phi[VREF_KMAX * 3], S[VREF_KMAX], J[VREF_KMAX * 3], dl;
  memset(J, 0, sizeof J);
  vref_flux_source(p, Q, J, Phi, S, &dl);
  equilibrium_from_flux(p, Q, Phi, feq);
}

/* Sec. 2.2 update with BGK collision and direct source injection (Sec. 3 intro):
 * zeroth and first moments Q_k = sum_i f_{k,i}, J_k = sum_i e_i f_{k,i};
 * fluxes and source from Q (and J for the div B estimate);
 * f*_{k,i} = f_{k,i} - (f_{k,i} - f^eq_{k,i}) / tau_k + w_i S~_k. */
static void homogenize(const vref_params* p, const int cell[3], double t, double* Q);

/* Moment matrix of the MRT collision (rows: 1, e_a, |e|^2, deviatoric second moments)
 * for the lattice, and its inverse by Gauss-Jordan elimination with partial pivoting. */
static void mrt_matrices(const vref_params* p, double Mm[7][7], double Mi[7][7]) {
  const int NQ = vref_ndirs(p), d = p->dim;
  for (int j = 0; j < 7; ++j)
    for (int i = 0; i < 7; ++i) Mm[j][i] = 0.0;
  for (int i = 0; i < NQ; ++i) {
    double e2[3] = {0.0, 0.0, 0.0}, ee = 0.0;
    for (int a = 0; a < d; ++a) {
      e2[a] = (double)(edir(i, a) * edir(i, a));
      ee += e2[a];
      Mm[1 + a][i] = edir(i, a);
    }
    Mm[0][i] = 1.0;
    Mm[1 + d][i] = ee;
    Mm[2 + d][i] = e2[0] - e2[1];
    if (d == 3) Mm[3 + d][i] = e2[0] + e2[1] - 2.0 * e2[2];
  }
  double A[7][14];
  for (int r = 0; r < NQ; ++r)
    for (int c = 0; c < 2 * NQ; ++c) A[r][c] = c < NQ ? Mm[r][c] : (c - NQ == r ? 1.0 : 0.0);
  for (int c = 0; c < NQ; ++c) {
    int piv = c;
    for (int r = c + 1; r < NQ; ++r)
      if (fabs(A[r][c]) > fabs(A[piv][c])) piv = r;
    for (int j = 0; j < 2 * NQ; ++j) {
      const double t = A[c][j];
      A[c][j] = A[piv][j];
      A[piv][j] = t;
    }
    const double inv = 1.0 / A[c][c];
    for (int j = 0; j < 2 * NQ; ++j) A[c][j] *= inv;
    for (int r = 0; r < NQ; ++r) {
      if (r == c) continue;
      const double fac = A[r][c];
      for (int j = 0; j < 2 * NQ; ++j) A[r][j] -= fac * A[c][j];
    }
  }
  for (int r = 0; r < NQ; ++r)
    for (int c = 0; c < NQ; ++c) Mi[r][c] = A[r][NQ + c];
}

/* Relaxation rate of the zeroth moment of variable k under the collision in use (TRT:
 * the symmetric rate 1/tau+_k, tau+ fixed by the magic parameter). */
static double zeroth_rate(const vref_params* p, int k) {
  switch (p->collision) {
    case 1: return 1.0 / (0.5 + p->trt_magic / (p->tau[k] - 0.5));
    case 2: return 1.0;
    case 3: return 1.0 / p->mrt_tau_e;
    default: return 1.0 / p->tau[k];
  }
}

/* Guo's state (Sec. 2.2 names the Guo source scheme; READING): Q = m + S~(Q)/2 with
 * m = sum_i f, solved by two fixed-point iterations Q0 = m + S~(m)/2,
 * Q = m + S~(Q0)/2 (second order in time for the source). */
static void guo_state(const vref_params* p, const double* m, const double* J, double* Q) {
  const int K = vref_nvars(p);
  double Phi[VREF_KMAX * 3], S[VREF_KMAX], dl, Q0[VREF_KMAX];
  vref_flux_source(p, m, J, Phi, S, &dl);
  for (int k = 0; k < K; ++k) Q0[k] = m[k] + 0.5 * S[k];
  vref_flux_source(p, Q0, J, Phi, S, &dl);
  for (int k = 0; k < K; ++k) Q[k] = m[k] + 0.5 * S[k];
}

/* cell == NULL: plain collision; else the cell's coordinates, and the target state
 * of the collision is homogenized with the body (Sec. 2.4) at time t.  sprev (K values,
 * Chai source only): the cell's source of the previous step, replaced by this step's. */
static int collide_cell(const vref_params* p, const double* f, double* fstar, double* dlat,
                        const int* cell, double t, double* sprev) {
  const int K = vref_nvars(p), NQ = vref_ndirs(p), d = p->dim;
  double Q[VREF_KMAX], J[VREF_KMAX * 3], Phi[VREF_KMAX * 3], S[VREF_KMAX];
  double feq[VREF_KMAX * 7];
  for (int k = 0; k < K; ++k) {
    Q[k] = 0.0;
    for (int a = 0; a < 3; ++a) J[3 * k + a] = 0.0;
    for (int i = 0; i < NQ; ++i) {
      Q[k] += f[k * NQ + i];
      for (int a = 0; a < d; ++a) J[3 * k + a] += edir(i, a) * f[k * NQ + i];
    }
  }
  if (p->source == 1) {
    double m[VREF_KMAX];
    for (int k = 0; k < K; ++k) m[k] = Q[k];
    guo_state(p, m, J, Q);
  }
  if (cell) homogenize(p, cell, t, Q);
  double dl;
  const int bad = vref_flux_source(p, Q, J, Phi, S, &dl);
  equilibrium_from_flux(p, Q, Phi, feq);
  /* the source as it enters the populations (w_i times this) */
  for (int k = 0; k < K; ++k) {
    if (p->source == 1) {
      S[k] *= 1.0 - 0.5 * zeroth_rate(p, k);
    } else if (p->source == 2) {
      /* without a stored previous source (a lone collision) the previous one is taken
       * equal to the current one, as at the start of a run */
      const double now = S[k];
      S[k] = now + 0.5 * (now - (sprev ? sprev[k] : now));
      if (sprev) sprev[k] = now;
    }
  }
  if (p->collision == 0) {
    for (int k = 0; k < K; ++k)
      for (int i = 0; i < NQ; ++i) {
        const double fo = f[k * NQ + i];
        fstar[k * NQ + i] = fo - (fo - feq[k * NQ + i]) / p->tau[k] + weight(p, i) * S[k];
      }
  } else if (p->collision == 1) {
    /* Sec. 2.2 names TRT among the admissible collisions.  READING: the
     * antisymmetric parts f^-_i = (f_i - f_ibar)/2 relax with 1/tau_k (they carry the
     * first moment, so tau_k keeps setting the transport), the symmetric parts
     * f^+_i = (f_i + f_ibar)/2 with 1/tau+_k, tau+ fixed by the magic parameter
     * Lambda = (tau+ - 1/2)(tau_k - 1/2). */
    for (int k = 0; k < K; ++k) {
      const double om_a = 1.0 / p->tau[k];
      const double om_s = zeroth_rate(p, k);
      for (int i = 0; i < NQ; ++i) {
        const int ib = i == 0 ? 0 : ((i % 2 == 1) ? i + 1 : i - 1);
        const double fp = 0.5 * (f[k * NQ + i] + f[k * NQ + ib]);
        const double fm = 0.5 * (f[k * NQ + i] - f[k * NQ + ib]);
        const double ep = 0.5 * (feq[k * NQ + i] + feq[k * NQ + ib]);
        const double em = 0.5 * (feq[k * NQ + i] - feq[k * NQ + ib]);
        fstar[k * NQ + i] = f[k * NQ + i] - om_s * (fp - ep) - om_a * (fm - em) + weight(p, i) * S[k];
      }
    }
  } else if (p->collision == 3) {
    /* Sec. 2.2 names MRT among the admissible collisions.  READING: the moments of
     * each variable's set are m = M f with the rows 1 (zeroth), e_a (first, one per
     * axis), |e|^2 (trace of the second moments) and the deviatoric second moments
     * e_x^2 - e_y^2 (and e_x^2 + e_y^2 - 2 e_z^2 in 3D); they relax toward
     * m^eq = M f^eq, the first moments at 1/tau_k (transport, as in BGK), the zeroth
     * moment and the trace at 1/mrt_tau_e, the deviatoric ones at 1/mrt_tau_d:
     * f* = f - M^-1 S M (f - f^eq) + w_i S~_k. */
    double Mm[7][7], Mi[7][7], rate[7];
    mrt_matrices(p, Mm, Mi);
    for (int j = 0; j < NQ; ++j) rate[j] = 0.0;
    for (int k = 0; k < K; ++k) {
      rate[0] = 1.0 / p->mrt_tau_e;
      for (int a = 0; a < d; ++a) rate[1 + a] = 1.0 / p->tau[k];
      rate[1 + d] = 1.0 / p->mrt_tau_e;
      for (int j = 2 + d; j < NQ; ++j) rate[j] = 1.0 / p->mrt_tau_d;
      double dm[7];
      for (int j = 0; j < NQ; ++j) {
        dm[j] = 0.0;
        for (int i = 0; i < NQ; ++i) dm[j] += Mm[j][i] * (f[k * NQ + i] - feq[k * NQ + i]);
        dm[j] *= rate[j];
      }
      for (int i = 0; i < NQ; ++i) {
        double df = 0.0;
        for (int j = 0; j < NQ; ++j) df += Mi[i][j] * dm[j];
        fstar[k * NQ + i] = f[k * NQ + i] - df + weight(p, i) * S[k];
      }
    }
  } else {
    /* Sec. 2.2 names the regularized BGK (RLB) among the admissible collisions: the
     * non-equilibrium part is replaced by its projection on the first-order Hermite
     * term, f^neq_i -> w_i e_i . J^neq / c_s^2 with J^neq = sum_i e_i (f_i - f^eq_i),
     * then relaxed: f* = f^eq + (1 - 1/tau_k) f^neq_reg + w_i S~_k. */
    const double c2 = cs2(p);
    for (int k = 0; k < K; ++k) {
      double Jn[3] = {0.0, 0.0, 0.0};
      for (int i = 0; i < NQ; ++i)
        for (int a = 0; a < d; ++a) Jn[a] += edir(i, a) * (f[k * NQ + i] - feq[k * NQ + i]);
      for (int i = 0; i < NQ; ++i) {
        double eJ = 0.0;
        for (int a = 0; a < d; ++a) eJ += edir(i, a) * Jn[a];
        const double fneq = weight(p, i) * eJ / c2;
        fstar[k * NQ + i] = feq[k * NQ + i] + (1.0 - 1.0 / p->tau[k]) * fneq + weight(p, i) * S[k];
      }
    }
  }
  if (dlat) *dlat = dl;
  return bad;
}

int vref_collide(const vref_params* p, const double* f, double* fstar, double* dlat) {
  return collide_cell(p, f, fstar, dlat, NULL, 0.0, NULL);
}

/* vref_collide on n independent cells: f and fstar are [n][K][Q]. */
int vref_collide_many(const vref_params* p, long n, const double* f, double* fstar) {
  const int KQ = vref_nvars(p) * vref_ndirs(p);
  int nbad = 0;
#pragma omp parallel for schedule(static) reduction(+ : nbad)
  for (long j = 0; j < n; ++j) nbad += vref_collide(p, f + j * KQ, fstar + j * KQ, NULL);
  return nbad;
}

int vref_collide_at(const vref_params* p, long n, const double* f, const int* xyz, double t, double* fstar) {
  const int KQ = vref_nvars(p) * vref_ndirs(p);
  int nbad = 0;
#pragma omp parallel for schedule(static) reduction(+ : nbad)
  for (long j = 0; j < n; ++j)
    nbad += collide_cell(p, f + j * KQ, fstar + j * KQ, NULL, p->body == 2 ? xyz + 3 * j : NULL, t, NULL);
  return nbad;
}

static long ncells(const vref_params* p) { return (long)p->nx * p->ny * p->nz; }

/* periodic neighbour of cell (x,y,z) along direction i */
static long neighbour(const vref_params* p, int x, int y, int z, int i) {
  int c[3] = {x, y, z};
  const int n[3] = {p->nx, p->ny, p->nz};
  for (int a = 0; a < p->dim; ++a) c[a] = ((c[a] + edir(i, a)) % n[a] + n[a]) % n[a];
  return (long)c[0] + (long)p->nx * ((long)c[1] + (long)p->ny * c[2]);
}

/* READING (initial populations, P7): f = f^eq(Q); with Guo's source the populations'
 * sum is the state minus half its source, sum_i f = Q - S~(Q)/2, the inverse of Guo's
 * half-source shift: f = f^eq(Q) - w_i S~(Q)/2. */
int vref_init(const vref_params* p, const double* Q, double* f) {
  const int K = vref_nvars(p), NQ = vref_ndirs(p);
  const long N = ncells(p);
#pragma omp parallel for schedule(static)
  for (long c = 0; c < N; ++c) {
    double q[VREF_KMAX], feq[VREF_KMAX * 7], Phi[VREF_KMAX * 3], S[VREF_KMAX], J[VREF_KMAX * 3], dl;
    for (int k = 0; k < K; ++k) q[k] = Q[k * N + c];
    vref_equilibrium(p, q, feq);
    if (p->source == 1) {
      memset(J, 0, sizeof J);
      vref_flux_source(p, q, J, Phi, S, &dl);
      for (int k = 0; k < K; ++k)
        for (int i = 0; i < NQ; ++i) feq[k * NQ + i] -= 0.5 * weight(p, i) * S[k];
    }
    for (int k = 0; k < K; ++k)
      for (int i = 0; i < NQ; ++i) f[((long)k * NQ + i) * N + c] = feq[k * NQ + i];
  }
  return 0;
}

/* Sec. 2.2 update: collide every cell, then push f*_{k,i}(x) to x + e_i (periodic). */
int vref_run(const vref_params* p, double* f, double* work, int nsteps) {
  return vref_run_src(p, f, work, NULL, nsteps);
}

int vref_run_src(const vref_params* p, double* f, double* work, double* sprev, int nsteps) {
  const int K = vref_nvars(p), NQ = vref_ndirs(p);
  const long N = ncells(p);
  if (p->source == 2 && !sprev) return -1;
  int nbad = 0;
  for (int step = 0; step < nsteps; ++step) {
#pragma omp parallel for collapse(2) schedule(static) reduction(+ : nbad)
    for (int z = 0; z < p->nz; ++z)
      for (int y = 0; y < p->ny; ++y)
        for (int x = 0; x < p->nx; ++x) {
          const long c = (long)x + (long)p->nx * ((long)y + (long)p->ny * z);
          double fc[VREF_KMAX * 7], fs[VREF_KMAX * 7];
          for (int k = 0; k < K; ++k)
            for (int i = 0; i < NQ; ++i) fc[k * NQ + i] = f[((long)k * NQ + i) * N + c];
          double sp[VREF_KMAX];
          if (sprev)
            for (int k = 0; k < K; ++k) sp[k] = sprev[(long)k * N + c];
          nbad += collide_cell(p, fc, fs, NULL, NULL, 0.0, sprev ? sp : NULL);
          if (sprev)
            for (int k = 0; k < K; ++k) sprev[(long)k * N + c] = sp[k];
          for (int i = 0; i < NQ; ++i) {
            const long t = neighbour(p, x, y, z, i);
            for (int k = 0; k < K; ++k) work[((long)k * NQ + i) * N + t] = fs[k * NQ + i];
          }
        }
    memcpy(f, work, sizeof(double) * (size_t)K * NQ * N);
  }
  return nbad;
}

int vref_source_field(const vref_params* p, const double* f, double* S_out) {
  const int K = vref_nvars(p), NQ = vref_ndirs(p), d = p->dim;
  const long N = ncells(p);
#pragma omp parallel for schedule(static)
  for (long c = 0; c < N; ++c) {
    double q[VREF_KMAX], J[VREF_KMAX * 3], Phi[VREF_KMAX * 3], S[VREF_KMAX], dl;
    for (int k = 0; k < K; ++k) {
      q[k] = 0.0;
      for (int a = 0; a < 3; ++a) J[3 * k + a] = 0.0;
      for (int i = 0; i < NQ; ++i) {
        const double v = f[((long)k * NQ + i) * N + c];
        q[k] += v;
        for (int a = 0; a < d; ++a) J[3 * k + a] += edir(i, a) * v;
      }
    }
    if (p->source == 1) {
      double m[VREF_KMAX];
      for (int k = 0; k < K; ++k) m[k] = q[k];
      guo_state(p, m, J, q);
    }
    vref_flux_source(p, q, J, Phi, S, &dl);
    for (int k = 0; k < K; ++k) S_out[(long)k * N + c] = S[k];
  }
  return 0;
}

int vref_moments(const vref_params* p, const double* f, double* Q_out, double* dlat,
                 double* totals) {
  const int K = vref_nvars(p), NQ = vref_ndirs(p), d = p->dim;
  const long N = ncells(p);
  double* Qall = (double*)malloc(sizeof(double) * (size_t)K * N);
  double* dall = (double*)malloc(sizeof(double) * (size_t)N);
  if (!Qall || !dall) {
    free(Qall);
    free(dall);
    return -1;
  }
  int nbad = 0;
#pragma omp parallel for schedule(static) reduction(+ : nbad)
  for (long c = 0; c < N; ++c) {
    double q[VREF_KMAX], J[VREF_KMAX * 3], Phi[VREF_KMAX * 3], S[VREF_KMAX], dl;
    for (int k = 0; k < K; ++k) {
      q[k] = 0.0;
      for (int a = 0; a < 3; ++a) J[3 * k + a] = 0.0;
      for (int i = 0; i < NQ; ++i) {
        const double v = f[((long)k * NQ + i) * N + c];
        q[k] += v;
        for (int a = 0; a < d; ++a) J[3 * k + a] += edir(i, a) * v;
      }
    }
    if (p->source == 1) {
      double m[VREF_KMAX];
      for (int k = 0; k < K; ++k) m[k] = q[k];
      guo_state(p, m, J, q);
    }
    for (int k = 0; k < K; ++k) Qall[(long)k * N + c] = q[k];
    nbad += vref_flux_source(p, q, J, Phi, S, &dl);
    dall[c] = dl;
  }
  if (totals) {
    for (int k = 0; k < K + 5; ++k) totals[k] = 0.0;
    for (int k = 0; k < K; ++k)
      for (long c = 0; c < N; ++c) totals[k] += Qall[(long)k * N + c];
    for (long c = 0; c < N; ++c) {
      totals[K] += dall[c];
      totals[K + 1] += dall[c] * dall[c];
      if (fabs(dall[c]) > totals[K + 2]) totals[K + 2] = fabs(dall[c]);
    }
    /* central-difference divergence of the moment field B, lattice units */
    for (int z = 0; z < (p->model == 2 || p->model == 3 ? 0 : p->nz); ++z)
      for (int y = 0; y < p->ny; ++y)
        for (int x = 0; x < p->nx; ++x) {
          double dv = 0.0;
          for (int a = 0; a < d; ++a) {
            const long cp = neighbour(p, x, y, z, 2 * a + 1);
            const long cm = neighbour(p, x, y, z, 2 * a + 2);
            dv += 0.5 * (Qall[(long)(bx_index(p) + a) * N + cp] - Qall[(long)(bx_index(p) + a) * N + cm]);
          }
          totals[K + 3] += dv * dv;
        }
    totals[K + 4] = nbad;
  }
  if (Q_out) memcpy(Q_out, Qall, sizeof(double) * (size_t)K * N);
  if (dlat) memcpy(dlat, dall, sizeof(double) * (size_t)N);
  free(Qall);
  free(dall);
  return nbad;
}

/* ------------------------------------------------------------------------- */
/* boundaries (Sec. 2.4) and the moving body                                 */
/* ------------------------------------------------------------------------- */

/* READING (body, not in the paper -- the paper uses a homogenised body): a rough
 * sphere given by its surface radius along each direction; solid = cell centre
 * strictly inside. */
/* Offset r of cell (x, y, z) from the body centre at time t, its length, and the
 * surface radius R0 (1 + delta(n)) along n = r / |r| (R0 at the centre). */
static double surface_radius(const vref_params* p, int x, int y, int z, double t, double r[3], double* rr) {
  r[0] = x - (p->body_c0[0] + t * p->body_v[0]);
  r[1] = y - (p->body_c0[1] + t * p->body_v[1]);
  r[2] = z - (p->body_c0[2] + t * p->body_v[2]);
  *rr = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  if (*rr == 0.0) return p->body_R0;
  double delta = 0.0;
  for (int j = 0; j < 4; ++j) {
    double dn = 0.0, en = 0.0;
    for (int a = 0; a < 3; ++a) {
      dn += p->body_d[j][a] * r[a] / *rr;
      en += p->body_e[j][a] * r[a] / *rr;
    }
    delta += p->body_a[j] * dn + p->body_b[j] * (en * en - 1.0 / 3.0);
  }
  return p->body_R0 * (1.0 + delta);
}

int vref_solid(const vref_params* p, int x, int y, int z, double t) {
  if (!p->body) return 0;
  double r[3], rr;
  const double R = surface_radius(p, x, y, z, t, r, &rr);
  return rr == 0.0 || rr < R;
}

/* Sec. 2.4 homogenization: lattice porosity d from the signed distance phi to the
 * surface (positive in the fluid) with the linear transition of width eps_h:
 * d = 0 for phi <= -eps_h/2, phi/eps_h + 1/2 inside, 1 for phi >= eps_h/2.
 * READING: eps_h = one cell (the paper's single-cell transition); phi = |r| - R(n),
 * the radial distance to the surface (exact for a sphere). */
double vref_porosity(const vref_params* p, int x, int y, int z, double t) {
  if (!p->body) return 1.0;
  double r[3], rr;
  const double R = surface_radius(p, x, y, z, t, r, &rr);
  const double phi = rr - R, eps = 1.0;
  if (phi <= -0.5 * eps) return 0.0;
  if (phi >= 0.5 * eps) return 1.0;
  return phi / eps + 0.5;
}

/* Field of the body at cell (x, y, z), time t.  READING (the paper gives the body a
 * prescribed field B^B without a formula): a sphere of radius R0 magnetised
 * uniformly with moment m -- the dipole field (3 (m.r) r - m |r|^2) / |r|^5
 * outside R0 and the uniform 2 m / R0^3 inside, which join with continuous normal
 * component, so that B^B is divergence free. */
static void body_field(const vref_params* p, int x, int y, int z, double t, double B[3]) {
  double r[3];
  r[0] = x - (p->body_c0[0] + t * p->body_v[0]);
  r[1] = y - (p->body_c0[1] + t * p->body_v[1]);
  r[2] = z - (p->body_c0[2] + t * p->body_v[2]);
  const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
  const double R0 = p->body_R0;
  if (r2 < R0 * R0) {
    for (int a = 0; a < 3; ++a) B[a] = 2.0 * p->body_m[a] / (R0 * R0 * R0);
    return;
  }
  const double r5 = r2 * r2 * sqrt(r2);
  const double mr = p->body_m[0] * r[0] + p->body_m[1] * r[1] + p->body_m[2] * r[2];
  for (int a = 0; a < 3; ++a) B[a] = (3.0 * mr * r[a] - p->body_m[a] * r2) / r5;
}

/* Sec. 2.4 homogenized target state of a cell: u^ = d u + (1 - d) u^B and
 * B^ = d B + (1 - d) B^B replace u and B in the equilibrium and the flux (and, as
 * a READING, in the Powell source evaluated with them).  READING: the homogenized
 * state keeps rho and the fluid's pressure, so e_tot^ = p/(gamma-1) + rho|u^|^2/2 +
 * |B^|^2/2.  u^B: the body's velocity in flux units, body_v / s (a velocity u moves
 * u s cells per step). */
static void homogenize(const vref_params* p, const int cell[3], double t, double* Q) {
  const double d = vref_porosity(p, cell[0], cell[1], cell[2], t);
  if (d >= 1.0) return;
  double Bb[3];
  body_field(p, cell[0], cell[1], cell[2], t, Bb);
  const double rho = Q[0], gm1 = p->gamma - 1.0;
  double u[3], uu = 0.0, BB = 0.0;
  for (int a = 0; a < 3; ++a) {
    u[a] = Q[1 + a] / rho;
    uu += u[a] * u[a];
    BB += Q[5 + a] * Q[5 + a];
  }
  const double pres = gm1 * (Q[4] - 0.5 * rho * uu - 0.5 * BB);
  double uh2 = 0.0, Bh2 = 0.0;
  for (int a = 0; a < 3; ++a) {
    const double uh = d * u[a] + (1.0 - d) * p->body_v[a] / p->s;
    const double Bh = d * Q[5 + a] + (1.0 - d) * Bb[a];
    Q[1 + a] = rho * uh;
    Q[5 + a] = Bh;
    uh2 += uh * uh;
    Bh2 += Bh * Bh;
  }
  Q[4] = pres / gm1 + 0.5 * rho * uh2 + 0.5 * Bh2;
}

/* dipole field of the body at point q (absolute cell coordinates), time t */
static void dipole_field(const vref_params* p, const double* q, double t, double* B) {
  double r[3];
  for (int a = 0; a < 3; ++a) r[a] = q[a] - (p->body_c0[a] + t * p->body_v[a]);
  const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
  const double r5 = r2 * r2 * sqrt(r2);
  const double mr = p->body_m[0] * r[0] + p->body_m[1] * r[1] + p->body_m[2] * r[2];
  for (int a = 0; a < 3; ++a) B[a] = (3.0 * mr * r[a] - p->body_m[a] * r2) / r5;
}

/* 1 if the cell lies on a non-periodic face; *inflow set if on an inflow face */
static int face_node(const vref_params* p, const int c[3], int* inflow) {
  const int n[3] = {p->nx, p->ny, p->nz};
  int on = 0;
  *inflow = 0;
  for (int a = 0; a < p->dim; ++a) {
    if (c[a] == 0 && p->bc[2 * a] != 0) {
      on = 1;
      if (p->bc[2 * a] == 1) *inflow = 1;
    }
    if (c[a] == n[a] - 1 && p->bc[2 * a + 1] != 0) {
      on = 1;
      if (p->bc[2 * a + 1] == 1) *inflow = 1;
    }
  }
  return on;
}

static void cell_moments(const vref_params* p, const double* f, long N, long cell, double* Q) {
  const int K = vref_nvars(p), NQ = vref_ndirs(p);
  for (int k = 0; k < K; ++k) {
    Q[k] = 0.0;
    for (int i = 0; i < NQ; ++i) Q[k] += f[((long)k * NQ + i) * N + cell];
  }
}

static long cell_index(const vref_params* p, const int c[3]) {
  return (long)c[0] + (long)p->nx * ((long)c[1] + (long)p->ny * c[2]);
}

int vref_run_bc(const vref_params* p, double* f, double* work, int nsteps, int t0) {
  const int K = vref_nvars(p), NQ = vref_ndirs(p), d = p->dim;
  const long N = ncells(p);
  const int n[3] = {p->nx, p->ny, p->nz};
  const double c2 = cs2(p), wi = weight(p, 1);
  unsigned char* solid = (unsigned char*)malloc((size_t)N);
  unsigned char* solid_next = (unsigned char*)malloc((size_t)N);
  double* qbc = (double*)malloc(sizeof(double) * (size_t)VREF_KMAX * N);
  if (!solid || !solid_next || !qbc) {
    free(solid);
    free(solid_next);
    free(qbc);
    return -1;
  }
  int nbad = 0;
  for (long c = 0; c < N; ++c) {
    const int x = (int)(c % p->nx), y = (int)((c / p->nx) % p->ny), z = (int)(c / ((long)p->nx * p->ny));
    solid[c] = (unsigned char)(p->body == 1 && vref_solid(p, x, y, z, (double)t0));
  }
  for (int step = 0; step < nsteps; ++step) {
    const double t = (double)(t0 + step);
    /* Sec. 2.4 static boundaries: every node on a non-periodic face takes the
     * equilibrium of its boundary state -- the Dirichlet state on an inflow face,
     * otherwise (zero gradient) the moments of the nearest interior cell along the
     * face normals.  All boundary states are read first, then written. */
    for (long cell = 0; cell < N; ++cell) {
      const int cc[3] = {(int)(cell % p->nx), (int)((cell / p->nx) % p->ny), (int)(cell / ((long)p->nx * p->ny))};
      int inflow;
      if (!face_node(p, cc, &inflow)) continue;
      double* Q = qbc + (long)VREF_KMAX * cell;
      if (inflow) {
        for (int k = 0; k < K; ++k) Q[k] = k < 8 ? p->inflow_Q[k] : 0.0;
      } else {
        int ic[3] = {cc[0], cc[1], cc[2]};
        for (int a = 0; a < d; ++a)
          if (p->bc[2 * a] != 0 || p->bc[2 * a + 1] != 0) {
            if (ic[a] < 1) ic[a] = 1;
            if (ic[a] > n[a] - 2) ic[a] = n[a] - 2;
          }
        cell_moments(p, f, N, cell_index(p, ic), Q);
      }
    }
    for (long cell = 0; cell < N; ++cell) {
      const int cc[3] = {(int)(cell % p->nx), (int)((cell / p->nx) % p->ny), (int)(cell / ((long)p->nx * p->ny))};
      int inflow;
      if (!face_node(p, cc, &inflow)) continue;
      double feq[VREF_KMAX * 7];
      vref_equilibrium(p, qbc + (long)VREF_KMAX * cell, feq);
      for (int k = 0; k < K; ++k)
        for (int i = 0; i < NQ; ++i) f[((long)k * NQ + i) * N + cell] = feq[k * NQ + i];
    }
    memset(work, 0, sizeof(double) * (size_t)K * NQ * N);
#pragma omp parallel for schedule(static) reduction(+ : nbad)
    for (long cell = 0; cell < N; ++cell) {
      if (solid[cell]) continue;
      const int cc[3] = {(int)(cell % p->nx), (int)((cell / p->nx) % p->ny), (int)(cell / ((long)p->nx * p->ny))};
      double fc[VREF_KMAX * 7], fs[VREF_KMAX * 7], Q[VREF_KMAX];
      for (int k = 0; k < K; ++k)
        for (int i = 0; i < NQ; ++i) fc[k * NQ + i] = f[((long)k * NQ + i) * N + cell];
      nbad += collide_cell(p, fc, fs, NULL, p->body == 2 ? cc : NULL, t, NULL);
      cell_moments(p, f, N, cell, Q);
      for (int k = 0; k < K; ++k) work[((long)k * NQ + 0) * N + cell] = fs[k * NQ + 0];
      for (int i = 1; i < NQ; ++i) {
        /* streaming with periodic addressing: what leaves through a non-periodic
         * face lands on a node of the opposite face, which the next step overwrites */
        const long tgt = neighbour(p, cc[0], cc[1], cc[2], i);
        const int ib = (i % 2 == 1) ? i + 1 : i - 1; /* opposite direction */
        if (solid[tgt]) {
          /* READING (body boundary): bounce back into the opposite direction of the
           * same cell.  rho, e_tot: halfway bounce-back with the moving-wall flux
           * correction -2 w_i c_i . s Phi_w / c_s^2 (Phi_w: the cell's flux with the
           * wall velocity); rho u, B: anti-bounce-back -f* + 2 w_i Q_w to the wall
           * values rho u_w and the dipole field at the link midpoint. */
          /* wall velocity in flux units: the body moves body_v cells per step,
           * a velocity u moves u s cells per step (s = dt/dx) */
          const double uw[3] = {p->body_v[0] / p->s, p->body_v[1] / p->s, p->body_v[2] / p->s};
          double q[3], Bw[3];
          for (int a = 0; a < 3; ++a) q[a] = cc[a] + 0.5 * (a < d ? edir(i, a) : 0);
          dipole_field(p, q, t, Bw);
          const double rho = Q[0], E = Q[4];
          const double B[3] = {Q[5], Q[6], Q[7]};
          double uu = 0.0, BB = 0.0;
          for (int a = 0; a < 3; ++a) {
            const double u = Q[1 + a] / rho;
            uu += u * u;
            BB += B[a] * B[a];
          }
          const double pcell = (p->gamma - 1.0) * (E - 0.5 * rho * uu - 0.5 * BB);
          const double ptcell = pcell + 0.5 * BB;
          const double uB = uw[0] * B[0] + uw[1] * B[1] + uw[2] * B[2];
          double ephi_rho = 0.0, ephi_E = 0.0;
          for (int a = 0; a < d; ++a) {
            ephi_rho += edir(i, a) * p->s * rho * uw[a];
            ephi_E += edir(i, a) * p->s * ((E + ptcell) * uw[a] - B[a] * uB);
          }
          for (int k = 0; k < K; ++k) {
            const double v = fs[k * NQ + i];
            double out;
            if (k == 0)
              out = v - 2.0 * wi * ephi_rho / c2;
            else if (k == 4)
              out = v - 2.0 * wi * ephi_E / c2;
            else if (k >= 1 && k <= 3)
              out = -v + 2.0 * wi * rho * uw[k - 1];
            else if (k >= 5 && k <= 7)
              out = -v + 2.0 * wi * Bw[k - 5];
            else
              out = v;
            work[((long)k * NQ + ib) * N + cell] = out;
          }
        } else {
          for (int k = 0; k < K; ++k) work[((long)k * NQ + i) * N + tgt] = fs[k * NQ + i];
        }
      }
    }
    memcpy(f, work, sizeof(double) * (size_t)K * NQ * N);
    /* body moves: cells it uncovers get f^eq of the mean moments of the neighbours
     * that are fluid before and after the move */
    for (long c = 0; c < N; ++c) {
      const int x = (int)(c % p->nx), y = (int)((c / p->nx) % p->ny), z = (int)(c / ((long)p->nx * p->ny));
      solid_next[c] = (unsigned char)(p->body == 1 && vref_solid(p, x, y, z, t + 1.0));
    }
    for (long c = 0; c < N; ++c) {
      if (!(solid[c] && !solid_next[c])) continue;
      const int cc[3] = {(int)(c % p->nx), (int)((c / p->nx) % p->ny), (int)(c / ((long)p->nx * p->ny))};
      double Qm[VREF_KMAX], Qn[VREF_KMAX];
      int cnt = 0;
      for (int k = 0; k < K; ++k) Qm[k] = 0.0;
      for (int i = 1; i < NQ; ++i) {
        const long nb = neighbour(p, cc[0], cc[1], cc[2], i);
        if (solid[nb] || solid_next[nb]) continue;
        cell_moments(p, f, N, nb, Qn);
        for (int k = 0; k < K; ++k) Qm[k] += Qn[k];
        ++cnt;
      }
      if (cnt == 0) {
        for (int k = 0; k < K; ++k) Qm[k] = k < 8 ? p->inflow_Q[k] : 0.0;
      } else {
        for (int k = 0; k < K; ++k) Qm[k] /= cnt;
      }
      double feq[VREF_KMAX * 7];
      vref_equilibrium(p, Qm, feq);
      for (int k = 0; k < K; ++k)
        for (int i = 0; i < NQ; ++i) f[((long)k * NQ + i) * N + c] = feq[k * NQ + i];
    }
    memcpy(solid, solid_next, (size_t)N);
  }
  free(solid);
  free(solid_next);
  free(qbc);
  return nbad;
}

// Per-cell physics of the VLBM MHD sweep: state -> flux, sources, div B estimate,
// and the BGK collision with direct source injection.  Host and device.
//
// Paper: "Lattice Boltzmann Methods for Compressible (Magneto)hydrodynamics".
//  - Sec. 2.2: update f_{k,i}(x + c_i, t + 1) = f_{k,i} + Omega^C + Omega^S, linear
//    vector equilibrium f^eq_{k,i} = w_i (Q_k + c_i . Phi_k / c_s^2), moments
//    Q_k = sum_i f_{k,i}.
//  - Sec. 2.3: ideal MHD state/flux, equation of state, Powell source; the expanded
//    resistive state with transported gradients (Sec. 2.2.1).
//  - Sec. 3 intro: BGK collision, direct injection of the source.
#pragma once

#include <hip/hip_runtime.h>

namespace vlbm {

constexpr int KMAX = 26;

// Direction i: 0 rest, 2a+1 is +e_a, 2a+2 is -e_a.
__host__ __device__ constexpr int opposite(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

// Model constants, converted to the compute type R by the kernel.
struct Phys {
  double s;          // flux scale dt/dx
  double gm1;        // gamma - 1
  double inv_cs2;    // 1 / c_s^2
  double w0, wi;     // rest and moving weights
  double omega[KMAX];// 1 / tau_k
  double inv_tauB[3];// 1 / tau of the B_x, B_y, B_z sets (div B estimate)
  double dt_over_tauM, dt_over_tauH;
  double mu, eta0, inv_jc2, inv_tauM, inv_tauH;
  double divb_scale; // divb_mode 1: dx = dt / s (lattice units of tr G / tau_M)
  int powell, divb_mode;
  int collision;     // 0 BGK; else the first moments (antisymmetric halves) at omega, the
                     // zeroth moment and the trace of the second moments at omega_s, their
                     // deviatoric part at omega_d (TRT and RLB: omega_d = omega_s; MRT apart)
  double omega_s[KMAX];
  double omega_d[KMAX];
  int source;        // 0 direct injection; 1 Guo (state = sum f + S/2, source times
                     // 1 - omega_0/2); 2 Chai (source + half its change since the last step)
  double lame_lambda, lame_mu, inv_rho0;  // Navier-Cauchy medium
};

// Number of conserved variables of a model: 8 ideal MHD (rho, rho u, E, B), 26
// resistive MHD (+ G, H), 5 compressible Euler (rho, rho u, E), 9 Navier-Cauchy
// (rho0 v, sigma_xx, yy, zz, xy, xz, yz).
// 13 for the 2D resistive system of Sec. 3.1 (rho, rho u_x, rho u_y, E, B_x, B_y, the
// transported stress xx xy yy and G xx xy yx yy).
template <int MODEL>
inline constexpr int kNVars = MODEL == 1 ? 26 : (MODEL == 2 ? 5 : (MODEL == 3 ? 9 : (MODEL == 4 ? 13 : 8)));
// Index of B_x in the state (models with a field).
template <int MODEL>
inline constexpr int kBx = MODEL == 4 ? 4 : 5;

// Index of sigma_bc in the Navier-Cauchy variables (symmetric, xx yy zz xy xz yz).
__host__ __device__ constexpr int sigma_index(int b, int c) {
  return b == c ? 3 + b : (b + c == 1 ? 6 : (b + c == 2 ? 7 : 8));
}

// Scaled lattice flux P[k][a] = (s / c_s^2) Phi[k][a] for the D lattice axes, lattice
// source S[k] and the lattice div B estimate.  Jb[a] = first moment along axis a of
// the B_a population set (only used by divb_mode 0).  Returns true if the cell is
// unphysical (rho <= 0, p < 0, or a non-finite value).
template <typename R, int D, int MODEL>
__host__ __device__ inline bool flux_source(const R* Q, const R* Jb, const Phys& ph,
                                            R (*P)[3], R* S, R& dlat, R* pt_out = nullptr) {
  constexpr int K = kNVars<MODEL>;
  if constexpr (MODEL == 4) {
    // The 13-component 2D system of Sec. 3.1 on D2Q5: the full flux of Sec. 2.3 with
    // the viscous stress carried as a transported stress T (xx, xy, yy) that settles
    // at tau_H mu (d_a u_b + d_b u_a) (its flux T u_c - mu (delta_ca u_b + delta_cb
    // u_a), its source -T dt / tau_H; tau_v = T / tau_H) and grad B as G / tau_M (G
    // xx, xy, yx, yy, flux G u_c - delta_ca B_b, source -G dt / tau_M); j = d_x B_y -
    // d_y B_x out of the plane.
    static_assert(D == 2, "the 13-component system is two-dimensional");
    const R rho = Q[0];
    const R ir = R(1) / rho;
    const R E = Q[3];
    const R u[2] = {Q[1] * ir, Q[2] * ir};
    const R B[2] = {Q[4], Q[5]};
    const R uu = u[0] * Q[1] + u[1] * Q[2];  // rho |u|^2
    const R bb = B[0] * B[0] + B[1] * B[1];
    const R ub = u[0] * B[0] + u[1] * B[1];
    const R pres = R(ph.gm1) * (E - R(0.5) * uu - R(0.5) * bb);
    const R pt = pres + R(0.5) * bb;
    if (pt_out) *pt_out = pt;
    const R itm = R(ph.inv_tauM), ith = R(ph.inv_tauH), muv = R(ph.mu);
    const R dB[2][2] = {{Q[9] * itm, Q[10] * itm}, {Q[11] * itm, Q[12] * itm}};
    const R tv[2][2] = {{Q[6] * ith, Q[7] * ith}, {Q[7] * ith, Q[8] * ith}};
    const R j = dB[0][1] - dB[1][0];
    R eta = R(ph.eta0);
    if (ph.inv_jc2 > 0.0) eta = eta * (R(1) + j * j * R(ph.inv_jc2));
    const R jxb[2] = {-j * B[1], j * B[0]};
    const R Ept = E + pt;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      P[0][c] = Q[1 + c];
      R utv = R(0);
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        P[1 + a][c] = Q[1 + a] * u[c] - B[a] * B[c] - tv[a][c] + (a == c ? pt : R(0));
        utv += u[a] * tv[a][c];
        P[4 + a][c] = u[c] * B[a] - B[c] * u[a] - eta * dB[c][a];
      }
      P[3][c] = Ept * u[c] - B[c] * ub - utv + eta * jxb[c];
      P[6][c] = Q[6] * u[c] - muv * (c == 0 ? R(2) * u[0] : R(0));                 // xx
      P[7][c] = Q[7] * u[c] - muv * (c == 0 ? u[1] : u[0]);                        // xy
      P[8][c] = Q[8] * u[c] - muv * (c == 1 ? R(2) * u[1] : R(0));                 // yy
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) P[9 + 2 * a + b][c] = Q[9 + 2 * a + b] * u[c] - (a == c ? B[b] : R(0));
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) S[k] = R(0);
    const R sh = R(-ph.dt_over_tauH), sg = R(-ph.dt_over_tauM);
#pragma unroll
    for (int q = 0; q < 3; ++q) S[6 + q] = Q[6 + q] * sh;
#pragma unroll
    for (int q = 0; q < 4; ++q) S[9 + q] = Q[9 + q] * sg;
    R divb;
    if (ph.divb_mode == 1) {
      divb = (dB[0][0] + dB[1][1]) * R(ph.divb_scale);
    } else {
      divb = -(Jb[0] * R(ph.inv_tauB[0]) + Jb[1] * R(ph.inv_tauB[1])) * R(ph.inv_cs2);
    }
    dlat = divb;
    if (ph.powell) {
      const R cp = -R(ph.s) * divb;
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        S[1 + b] += cp * B[b];
        S[4 + b] += cp * u[b];
      }
      S[3] += cp * ub;
    }
    const R c = R(ph.s * ph.inv_cs2);
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int a = 0; a < 2; ++a) P[k][a] *= c;
    bool bad = !(rho > R(0)) || !(pres >= R(0));
#pragma unroll
    for (int k = 0; k < K; ++k) bad = bad || !(Q[k] - Q[k] == R(0));
    return bad;
  } else if constexpr (MODEL == 3) {
    // linear Navier-Cauchy in velocity-stress form: the momentum flux is minus the
    // stress, the stress flux minus the isotropic (lambda) and shear (mu) rates of v
    (void)Jb;
    const R ir0 = R(ph.inv_rho0);
    const R v[3] = {Q[0] * ir0, Q[1] * ir0, Q[2] * ir0};
    const R lam = R(ph.lame_lambda), mu = R(ph.lame_mu);
    const R c = R(ph.s * ph.inv_cs2);
    if (pt_out) *pt_out = R(0);
#pragma unroll
    for (int a = 0; a < D; ++a) {
#pragma unroll
      for (int b = 0; b < 3; ++b) P[b][a] = -c * Q[sigma_index(b, a)];
#pragma unroll
      for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int cc = b; cc < 3; ++cc)
          P[sigma_index(b, cc)][a] = -c * ((b == cc ? lam * v[a] : R(0)) +
                                           mu * ((a == b ? v[cc] : R(0)) + (a == cc ? v[b] : R(0))));
    }
#pragma unroll
    for (int k = 0; k < K; ++k) S[k] = R(0);
    dlat = R(0);
    bool bad = false;
#pragma unroll
    for (int k = 0; k < K; ++k) bad = bad || !(Q[k] - Q[k] == R(0));
    return bad;
  } else if constexpr (MODEL == 2) {
    // compressible Euler: the ideal system without the field (the hydrodynamic limit
    // the paper's scheme covers, Sec. 1 and Sec. 2.3): mass, momentum, energy fluxes
    (void)Jb;
    const R rho = Q[0];
    const R ir = R(1) / rho;
    const R m[3] = {Q[1], Q[2], Q[3]};
    const R E = Q[4];
    const R u[3] = {m[0] * ir, m[1] * ir, m[2] * ir};
    const R pres = R(ph.gm1) * (E - R(0.5) * (m[0] * u[0] + m[1] * u[1] + m[2] * u[2]));
    const R c = R(ph.s * ph.inv_cs2);
    if (pt_out) *pt_out = pres;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      P[0][a] = c * m[a];
#pragma unroll
      for (int b = 0; b < 3; ++b) P[1 + b][a] = c * (m[b] * u[a] + (a == b ? pres : R(0)));
      P[4][a] = c * ((E + pres) * u[a]);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) S[k] = R(0);
    dlat = R(0);
    bool bad = !(rho > R(0)) || !(pres >= R(0));
#pragma unroll
    for (int k = 0; k < K; ++k) bad = bad || !(Q[k] - Q[k] == R(0));
    return bad;
  } else {
  const R rho = Q[0];
  const R ir = R(1) / rho;
  const R m0 = Q[1], m1 = Q[2], m2 = Q[3];
  const R E = Q[4];
  const R b0 = Q[5], b1 = Q[6], b2 = Q[7];
  const R u0 = m0 * ir, u1 = m1 * ir, u2 = m2 * ir;
  const R mu_ = m0 * u0 + m1 * u1 + m2 * u2;  // rho |u|^2
  const R bb = b0 * b0 + b1 * b1 + b2 * b2;
  const R ub = u0 * b0 + u1 * b1 + u2 * b2;
  const R pres = R(ph.gm1) * (E - R(0.5) * mu_ - R(0.5) * bb);
  const R pt = pres + R(0.5) * bb;
  const R c = R(ph.s * ph.inv_cs2);
  const R u[3] = {u0, u1, u2};
  const R m[3] = {m0, m1, m2};
  const R B[3] = {b0, b1, b2};
  const R Ept = E + pt;
  if (pt_out) *pt_out = pt;

  // physical fluxes along the lattice axes a (Sec. 2.3, ideal MHD)
#pragma unroll
  for (int a = 0; a < D; ++a) {
    P[0][a] = m[a];
#pragma unroll
    for (int b = 0; b < 3; ++b) P[1 + b][a] = m[b] * u[a] - B[b] * B[a] + (a == b ? pt : R(0));
    P[4][a] = Ept * u[a] - B[a] * ub;
#pragma unroll
    for (int b = 0; b < 3; ++b) P[5 + b][a] = u[a] * B[b] - B[a] * u[b];
  }
#pragma unroll
  for (int k = 0; k < K; ++k) S[k] = R(0);

  R divb;
  if constexpr (MODEL == 1) {
    // expanded state: G ~ tau_M grad B, H ~ tau_H grad u (Sec. 2.2.1, Sec. 2.3)
    const R* G = Q + 8;
    const R* H = Q + 17;
    const R itm = R(ph.inv_tauM), ith = R(ph.inv_tauH);
    R dB[3][3], du[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        dB[a][b] = G[3 * a + b] * itm;
        du[a][b] = H[3 * a + b] * ith;
      }
    const R j0 = dB[1][2] - dB[2][1], j1 = dB[2][0] - dB[0][2], j2 = dB[0][1] - dB[1][0];
    R eta = R(ph.eta0);
    if (ph.inv_jc2 > 0.0) eta = eta * (R(1) + (j0 * j0 + j1 * j1 + j2 * j2) * R(ph.inv_jc2));
    const R jxb[3] = {j1 * b2 - j2 * b1, j2 * b0 - j0 * b2, j0 * b1 - j1 * b0};
    const R muv = R(ph.mu);
#pragma unroll
    for (int a = 0; a < D; ++a) {
      R utv = R(0);
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const R tv = muv * (du[b][a] + du[a][b]);  // viscous stress, symmetric
        P[1 + b][a] -= tv;
        utv += u[b] * tv;
        P[5 + b][a] -= eta * dB[a][b];           // -eta d_a B_b in the flux of B_b
      }
      P[4][a] += eta * jxb[a] - utv;
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        const int ga = q / 3, gb = q % 3;
        P[8 + q][a] = G[q] * u[a] - (a == ga ? B[gb] : R(0));
        P[17 + q][a] = H[q] * u[a] - (a == ga ? u[gb] : R(0));
      }
    }
    const R sg = R(-ph.dt_over_tauM), sh = R(-ph.dt_over_tauH);
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      S[8 + q] = G[q] * sg;
      S[17 + q] = H[q] * sh;
    }
    if (ph.divb_mode == 1) {
      R tr = R(0);
#pragma unroll
      for (int a = 0; a < D; ++a) tr += dB[a][a];
      divb = tr * R(ph.divb_scale);
    } else {
      R acc = R(0);
#pragma unroll
      for (int a = 0; a < D; ++a) acc += Jb[a] * R(ph.inv_tauB[a]);
      divb = -acc * R(ph.inv_cs2);
    }
  } else {
    // local non-equilibrium estimate of div B from the B sets' first moments
    R acc = R(0);
#pragma unroll
    for (int a = 0; a < D; ++a) acc += Jb[a] * R(ph.inv_tauB[a]);
    divb = -acc * R(ph.inv_cs2);
  }
  dlat = divb;

  // Powell source -(div B)(0, B, u.B, u), times dt (= s times lattice divergence)
  if (ph.powell) {
    const R cp = -R(ph.s) * divb;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      S[1 + b] += cp * B[b];
      S[5 + b] += cp * u[b];
    }
    S[4] += cp * ub;
  }
  // scale the fluxes to c_i . Phi / c_s^2 units of the equilibrium
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int a = 0; a < D; ++a) P[k][a] *= c;

  bool bad = !(rho > R(0)) || !(pres >= R(0));
#pragma unroll
  for (int k = 0; k < K; ++k) bad = bad || !(Q[k] - Q[k] == R(0));  // NaN or Inf
  return bad;
  }
}

// Rest weight derived in the compute type as 1 - 2 D w_i, so that the weights sum
// to exactly one in that type: with w0 and w_i rounded independently (1/3 and 1/6
// in FP32 sum to 1 + 3e-8) the equilibrium would create mass every step.
template <typename R, int D>
__host__ __device__ inline R rest_weight(R wi) {
  return R(1) - R(2 * D) * wi;
}

// Equilibrium of one variable: f^eq_i = w_i (Q + c_i . P) with P already scaled.
template <typename R, int D>
__host__ __device__ inline R feq_dir(R Qk, const R* Pk, int i, R w0, R wi) {
  if (i == 0) return w0 * Qk;
  const int a = (i - 1) >> 1;
  return (i & 1) ? wi * (Qk + Pk[a]) : wi * (Qk - Pk[a]);
}

// Target of the collision: the state whose equilibrium, flux and source the
// populations relax toward.  NoTarget keeps the cell's own moments.
struct NoTarget {
  template <typename R>
  __device__ __forceinline__ void operator()(R*) const {}
};

// BGK + direct injection, in place: f_{k,i} += omega_k (f^eq_{k,i}(Q') - f_{k,i}) + w_i S_k(Q'),
// Q' the moments Q after tgt.  Returns the unphysical flag and writes the div B
// estimate, the pre-collision moments Q and the total pressure pt of Q'.
// COLL 0: BGK; 1: two relaxation rates (TRT, and the regularized BGK as its case
// omega_s = 1) -- a template parameter, so that the BGK sweep keeps its registers.
// SRC: the source operator (Sec. 2.2 names direct injection, Guo's and Chai's): 0 direct
// injection of w_i S~(Q); 1 Guo -- the state is Q = sum f + S~(Q)/2, found by two
// fixed-point iterations from the populations' sum, and the source enters as
// (1 - omega_0/2) w_i S~ with omega_0 the zeroth moment's rate; 2 Chai -- the source
// enters as w_i (S~ + (S~ - S~_prev)/2), sp holding the cell's S~_prev on entry and
// this step's S~ on return.
template <typename R, int D, int MODEL, int COLL = 0, typename Tgt = NoTarget, int SRC = 0>
__device__ __forceinline__ bool collide(R (*f)[2 * D + 1], const Phys& ph, R& dlat,
                                        R (&Q)[kNVars<MODEL>], R& pt, const Tgt& tgt = Tgt{},
                                        R* sp = nullptr) {
  constexpr int K = kNVars<MODEL>;
  // Zeroth moments, opposite directions paired first: f_{+a} + f_{-a} cancels the
  // flux part c_a . Phi / c_s^2 the two carry with opposite signs before it is
  // accumulated, which keeps small variables (G, H, a momentum at rest) accurate
  // in FP32.
#pragma unroll
  for (int k = 0; k < K; ++k) {
    R acc = f[k][0];
#pragma unroll
    for (int a = 0; a < D; ++a) acc += f[k][2 * a + 1] + f[k][2 * a + 2];
    Q[k] = acc;
  }
  R Jb[3] = {R(0), R(0), R(0)};
  if constexpr (MODEL == 0 || MODEL == 1 || MODEL == 4) {
    constexpr int bx = kBx<MODEL>;
#pragma unroll
    for (int a = 0; a < D; ++a) Jb[a] = f[bx + a][2 * a + 1] - f[bx + a][2 * a + 2];
  }
  R Qt[K];
#pragma unroll
  for (int k = 0; k < K; ++k) Qt[k] = Q[k];
  if constexpr (SRC == 1) {
    R P0[K][3], S0[K], d0;
    flux_source<R, D, MODEL>(Q, Jb, ph, P0, S0, d0);
#pragma unroll
    for (int k = 0; k < K; ++k) Qt[k] = Q[k] + R(0.5) * S0[k];
    flux_source<R, D, MODEL>(Qt, Jb, ph, P0, S0, d0);
#pragma unroll
    for (int k = 0; k < K; ++k) Qt[k] = Q[k] + R(0.5) * S0[k];
  }
  tgt(Qt);
  R P[K][3];
  R S[K];
  const bool bad = flux_source<R, D, MODEL>(Qt, Jb, ph, P, S, dlat, &pt);
  if constexpr (SRC == 1) {
#pragma unroll
    for (int k = 0; k < K; ++k) S[k] *= R(1) - R(0.5) * R(COLL == 0 ? ph.omega[k] : ph.omega_s[k]);
  } else if constexpr (SRC == 2) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const R now = S[k];
      S[k] = now + R(0.5) * (now - sp[k]);
      sp[k] = now;
    }
  }
  const R wi = R(ph.wi);
  const R w0 = rest_weight<R, D>(wi);
  if constexpr (COLL == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const R om = R(ph.omega[k]);
      const R sw0 = w0 * S[k], swi = wi * S[k];
      f[k][0] += om * (w0 * Qt[k] - f[k][0]) + sw0;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const R ep = wi * (Qt[k] + P[k][a]);
        const R em = wi * (Qt[k] - P[k][a]);
        f[k][2 * a + 1] += om * (ep - f[k][2 * a + 1]) + swi;
        f[k][2 * a + 2] += om * (em - f[k][2 * a + 2]) + swi;
      }
    }
  } else {
    // moment relaxation over each opposite pair: the antisymmetric half (f_+ - f_-)/2
    // (the first moment) toward w_i P at omega; the symmetric halves' non-equilibrium
    // parts h_a = (f_+ + f_-)/2 - w_i Q split into their mean over the axes (the trace
    // of the second moments), relaxed with the rest population at omega_s, and their
    // deviations from it, relaxed at omega_d.  omega_d = omega_s: TRT (and the
    // regularized BGK of these first-order lattices, omega_s = 1); else MRT.
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const R oa = R(ph.omega[k]), os = R(ph.omega_s[k]), od = R(ph.omega_d[k]);
      const R sw0 = w0 * S[k], swi = wi * S[k];
      f[k][0] += os * (w0 * Qt[k] - f[k][0]) + sw0;
      R h[D], hm = R(0);
#pragma unroll
      for (int a = 0; a < D; ++a) {
        h[a] = R(0.5) * (f[k][2 * a + 1] + f[k][2 * a + 2]) - wi * Qt[k];
        hm += h[a];
      }
      hm *= R(1.0 / D);
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const R fp = f[k][2 * a + 1], fm = f[k][2 * a + 2];
        const R ds = os * hm + od * (h[a] - hm);
        const R da = oa * (R(0.5) * (fp - fm) - wi * P[k][a]);
        f[k][2 * a + 1] = fp - ds - da + swi;
        f[k][2 * a + 2] = fm - ds + da + swi;
      }
    }
  }
  return bad;
}

template <typename R, int D, int MODEL, int COLL = 0>
__device__ __forceinline__ bool collide(R (*f)[2 * D + 1], const Phys& ph, R& dlat) {
  R Q[kNVars<MODEL>];
  R pt;
  return collide<R, D, MODEL, COLL>(f, ph, dlat, Q, pt);
}

}  // namespace vlbm

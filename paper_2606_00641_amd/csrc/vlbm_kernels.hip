// HIP kernels (gfx950) around the sweep: static faces, the body's mask and refill,
// init, moments and FP64 diagnostics, gather, conversions and the streaming copy.
// Population placement follows the sweep's in-place AA pattern (vlbm_sweep.hip):
// after an even number of steps f_i(x) sits at slot i of cell x, after an odd number
// at slot opposite(i) of cell x - e_i.
#include "vlbm_device.h"

namespace vlbm {
namespace {

// Population f_i of cell c in the layout of the given parity: its slot and the byte
// offset of the cell that holds it.
template <int D>
__device__ __forceinline__ void pop_place(int parity, int i, unsigned c, const unsigned (&np)[3],
                                          const unsigned (&nm)[3], int& slot, unsigned& cell) {
  slot = (parity == 0) ? i : opposite(i);
  cell = (parity == 0 || i == 0) ? c : ((i & 1) ? nm[(i - 1) >> 1] : np[(i - 1) >> 1]);
}

template <int ST>
__device__ inline void cell_moments3(const Grid& g, const Codec& cd, int parity, unsigned c,
                                     typename Store<ST>::R (&Q)[8]) {
  using S = Store<ST>;
  using T = typename S::T;
  using R = typename S::R;
  const int x = (int)(c % (unsigned)g.nx), y = (int)((c / (unsigned)g.nx) % (unsigned)g.ny);
  const int z = (int)(c / ((unsigned)g.nx * (unsigned)g.ny));
  unsigned np[3], nm[3];
  neighbours<3>(g, x, y, z, c, np, nm);
  const T* F = static_cast<const T*>(g.f);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    R q = R(0);
#pragma unroll
    for (int i = 0; i < 7; ++i) {
      int slot;
      unsigned src;
      pop_place<3>(parity, i, c, np, nm, slot, src);
      q += S::dec(F[(size_t)(k * 7 + slot) * g.stride + src], cd, k * 7 + i);
    }
    Q[k] = q;
  }
}

// f := f^eq(Q) for cell c in the layout of the given parity (D3Q7 ideal).
template <int ST>
__device__ inline void write_feq3(const Grid& g, const Phys& ph, const Codec& cd, int parity, unsigned c,
                                  const typename Store<ST>::R (&Q)[8]) {
  using S = Store<ST>;
  using T = typename S::T;
  using R = typename S::R;
  const int x = (int)(c % (unsigned)g.nx), y = (int)((c / (unsigned)g.nx) % (unsigned)g.ny);
  const int z = (int)(c / ((unsigned)g.nx * (unsigned)g.ny));
  unsigned np[3], nm[3];
  neighbours<3>(g, x, y, z, c, np, nm);
  R Jb[3] = {R(0), R(0), R(0)};
  R P[8][3], Sv[8], dl;
  flux_source<R, 3, 0>(Q, Jb, ph, P, Sv, dl);
  const R wi = R(ph.wi);
  const R w0 = rest_weight<R, 3>(wi);
  T* F = static_cast<T*>(g.f);
#pragma unroll
  for (int k = 0; k < 8; ++k)
#pragma unroll
    for (int i = 0; i < 7; ++i) {
      int slot;
      unsigned dst;
      pop_place<3>(parity, i, c, np, nm, slot, dst);
      F[(size_t)(k * 7 + slot) * g.stride + dst] = S::enc(feq_dir<R, 3>(Q[k], P[k], i, w0, wi), cd, k * 7 + i);
    }
}

// Static faces.  blockIdx.z is the face (2a + side); a thread per node of it.  A node
// on several non-periodic faces is handled by each of them with identical values (the
// x faces by the sweep itself where it can, see fuse_x_faces; their edges with the y
// and z faces still here);
// the cells read (no non-periodic face) and the populations written (face nodes
// only) are disjoint.
template <int ST>
__global__ __launch_bounds__(256) void k_faces(const Grid g, const Phys ph, const Codec cd, int parity,
                                               const Inflow in) {
  using R = typename Store<ST>::R;
  const int f = blockIdx.z, a = f >> 1;
  if (g.bc[f] == 0) return;
  if (a == 0 && fuse_x_faces(g)) return;  // the sweep re-sets these nodes
  const int n[3] = {g.nx, g.ny, g.nz};
  // the two other axes in increasing order, so that consecutive threads walk along x
  // (consecutive addresses) on the y and z faces
  const int a1 = a == 0 ? 1 : 0, a2 = a == 2 ? 1 : 2;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)n[a1] * n[a2]) return;
  int cc[3];
  cc[a] = (f & 1) ? n[a] - 1 : 0;
  cc[a1] = (int)(t % n[a1]);
  cc[a2] = (int)(t / n[a1]);
  bool inflow = false;
  int ic[3] = {cc[0], cc[1], cc[2]};
  for (int b = 0; b < 3; ++b) {
    if (g.bc[2 * b] == 0) continue;
    if ((cc[b] == 0 && g.bc[2 * b] == 1) || (cc[b] == n[b] - 1 && g.bc[2 * b + 1] == 1)) inflow = true;
    ic[b] = min(max(cc[b], 1), n[b] - 2);
  }
  R Q[8];
  if (inflow) {
#pragma unroll
    for (int k = 0; k < 8; ++k) Q[k] = R(in.q[k]);
  } else {
    cell_moments3<ST>(g, cd, parity, (unsigned)ic[0] + (unsigned)g.nx * ((unsigned)ic[1] + (unsigned)g.ny * ic[2]), Q);
  }
  write_feq3<ST>(g, ph, cd, parity, (unsigned)cc[0] + (unsigned)g.nx * ((unsigned)cc[1] + (unsigned)g.ny * cc[2]),
                 Q);
}

__device__ __forceinline__ bool box_cell(const Body& b, int& x, int& y, int& z) {
  const long long bx = b.box[1] - b.box[0], by = b.box[3] - b.box[2], bz = b.box[5] - b.box[4];
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= bx * by * bz) return false;
  x = b.box[0] + (int)(t % bx);
  y = b.box[2] + (int)((t / bx) % by);
  z = b.box[4] + (int)(t / (bx * by));
  return true;
}

// Mask pass 0 (solid bit at time b.t; the previous solid bit kept as kWasSolid unless
// fresh) and pass 1 (link bits from the neighbours' solid bits; only bits 1..6 of the
// own byte change, so concurrent reads of bit 7 are unaffected).
__global__ __launch_bounds__(256) void k_mask(const Grid g, const Body b, int pass, int fresh) {
  int x, y, z;
  if (!box_cell(b, x, y, z)) return;
  const unsigned c = (unsigned)x + (unsigned)g.nx * ((unsigned)y + (unsigned)g.ny * (unsigned)z);
  const unsigned old = g.mask[c];
  if (pass == 0) {
    unsigned v = body_solid(b, x, y, z, b.t) ? kSolid : 0u;
    if (!fresh && (old & kSolid)) v |= kWasSolid;
    g.mask[c] = (unsigned char)v;
  } else {
    unsigned np[3], nm[3];
    neighbours<3>(g, x, y, z, c, np, nm);
    unsigned v = old & (kSolid | kWasSolid);
#pragma unroll
    for (int i = 1; i < 7; ++i) {
      const unsigned nb = (i & 1) ? np[(i - 1) >> 1] : nm[(i - 1) >> 1];
      if (g.mask[nb] & kSolid) v |= link_bit(i);
    }
    g.mask[c] = (unsigned char)v;
  }
}

// Refill of uncovered cells.  The neighbours read are fluid before and after the
// move, so no cell that is read is also written.
template <int ST>
__global__ __launch_bounds__(256) void k_refill(const Grid g, const Phys ph, const Codec cd, int parity,
                                                const Body b, const Inflow in) {
  using R = typename Store<ST>::R;
  int x, y, z;
  if (!box_cell(b, x, y, z)) return;
  const unsigned c = (unsigned)x + (unsigned)g.nx * ((unsigned)y + (unsigned)g.ny * (unsigned)z);
  const unsigned m = g.mask[c];
  if (!(m & kWasSolid) || (m & kSolid)) return;
  unsigned np[3], nm[3];
  neighbours<3>(g, x, y, z, c, np, nm);
  R Qm[8], Qn[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) Qm[k] = R(0);
  int cnt = 0;
  for (int i = 1; i < 7; ++i) {
    const unsigned nb = (i & 1) ? np[(i - 1) >> 1] : nm[(i - 1) >> 1];
    if (g.mask[nb] & (kSolid | kWasSolid)) continue;
    cell_moments3<ST>(g, cd, parity, nb, Qn);
#pragma unroll
    for (int k = 0; k < 8; ++k) Qm[k] += Qn[k];
    ++cnt;
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) Qm[k] = cnt ? Qm[k] / R(cnt) : R(in.q[k]);
  write_feq3<ST>(g, ph, cd, parity, c, Qm);
}

// ---------------------------------------------------------------------------
// init: f := f^eq(Q), natural layout
// ---------------------------------------------------------------------------
template <int ST, int D, int MODEL, typename QT>
__global__ __launch_bounds__(256) void k_init(const Grid g, const Phys ph, const Codec cd,
                                              const QT* __restrict__ Qin) {
  using S = Store<ST>;
  using T = typename S::T;
  using R = typename S::R;
  constexpr int NQ = 2 * D + 1;
  constexpr int K = kNVars<MODEL>;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= g.nx) return;
  const unsigned c = (unsigned)x + (unsigned)g.nx * (blockIdx.y + (unsigned)g.ny * blockIdx.z);
  const size_t N = (size_t)g.nx * g.ny * g.nz;
  T* __restrict__ F = static_cast<T*>(g.f);
  R Q[K];
#pragma unroll
  for (int k = 0; k < K; ++k) Q[k] = (R)Qin[(size_t)k * N + c];
  R Jb[3] = {R(0), R(0), R(0)};
  R P[K][3], Sv[K], dl;
  flux_source<R, D, MODEL>(Q, Jb, ph, P, Sv, dl);
  const R wi = R(ph.wi);
  const R w0 = rest_weight<R, D>(wi);
  // Guo's source: the populations' sum is the state minus half its source (the inverse
  // of the sweep's half-source shift); Chai's: the previous source starts as S~(Q)
  const R gs = ph.source == 1 ? R(0.5) : R(0);
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int i = 0; i < NQ; ++i)
      F[pop_index(g, NQ, k, i, c)] =
          S::enc(feq_dir<R, D>(Q[k], P[k], i, w0, wi) - gs * (i == 0 ? w0 : wi) * Sv[k], cd, k * NQ + i);
  if (ph.source == 2 && g.sprev) {
#pragma unroll
    for (int k = 0; k < K; ++k) static_cast<R*>(g.sprev)[(size_t)k * N + c] = Sv[k];
  }
}

// ---------------------------------------------------------------------------
// reductions (FP64)
// ---------------------------------------------------------------------------
// Reduce v[0..n) over the block (slots in maxmask take the max, others the sum) and
// let thread j < n write the block result of slot j to out[j].  All threads call it.
template <int NMAX>
__device__ void block_reduce(double (&v)[NMAX], int n, unsigned maxmask, double* out) {
  __shared__ double sh[kReduceThreads / 64][NMAX];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int j = 0; j < n; ++j) {
    const bool mx = (maxmask >> j) & 1u;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double o = __shfl_xor(v[j], off);
      v[j] = mx ? fmax(v[j], o) : v[j] + o;
    }
    if (lane == 0) sh[wv][j] = v[j];
  }
  __syncthreads();
  if ((int)threadIdx.x < n) {
    const int j = threadIdx.x;
    const bool mx = (maxmask >> j) & 1u;
    double r = sh[0][j];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = mx ? fmax(r, sh[w][j]) : r + sh[w][j];
    out[j] = r;
  }
}

template <int ST, int D, int MODEL>
__global__ __launch_bounds__(kReduceThreads) void k_moments(const Grid g, const Phys ph,
                                                            const Codec cd, int parity,
                                                            double* __restrict__ Qout,
                                                            double* __restrict__ partial) {
  using S = Store<ST>;
  using T = typename S::T;
  constexpr int NQ = 2 * D + 1;
  constexpr int K = kNVars<MODEL>;
  constexpr int NT = K + 5;
  const T* __restrict__ F = static_cast<const T*>(g.f);
  const size_t N = (size_t)g.nx * g.ny * g.nz;
  double acc[NT];
#pragma unroll
  for (int j = 0; j < NT; ++j) acc[j] = 0.0;
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < N;
       c += (size_t)gridDim.x * blockDim.x) {
    const int x = (int)(c % g.nx);
    const int y = (int)((c / g.nx) % g.ny);
    const int z = (int)(c / ((size_t)g.nx * g.ny));
    if (g.mask && (g.mask[c] & kSolid)) {  // inside the body: no fluid state
#pragma unroll
      for (int k = 0; k < K; ++k) Qout[(size_t)k * N + c] = 0.0;
      continue;
    }
    unsigned np[3], nm[3];
    neighbours<D>(g, x, y, z, (unsigned)c, np, nm);
    double Q[K];
    double Jb[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double q = 0.0;
#pragma unroll
      for (int i = 0; i < NQ; ++i) {
        const unsigned src = (parity == 0 || i == 0) ? (unsigned)c
                             : ((i & 1) ? nm[(i - 1) >> 1] : np[(i - 1) >> 1]);
        const int slot = parity == 0 ? i : opposite(i);
        const double v = S::dec64(F[pop_index(g, NQ, k, slot, src)], cd, k * NQ + i);
        q += v;
        constexpr int bx = kBx<MODEL>;
        if (k >= bx && k < bx + D && i > 0 && ((i - 1) >> 1) == k - bx) Jb[k - bx] += (i & 1) ? v : -v;
      }
      Q[k] = q;
      Qout[(size_t)k * N + c] = q;
    }
    double P[K][3], Sv[K], dl;
    if (ph.source == 1) {
      // Guo's state: sum f + S~/2 by the sweep's two fixed-point iterations
      double q[K];
      flux_source<double, D, MODEL>(Q, Jb, ph, P, Sv, dl);
#pragma unroll
      for (int k = 0; k < K; ++k) q[k] = Q[k] + 0.5 * Sv[k];
      flux_source<double, D, MODEL>(q, Jb, ph, P, Sv, dl);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        Q[k] += 0.5 * Sv[k];
        Qout[(size_t)k * N + c] = Q[k];
      }
    }
    const bool bad = flux_source<double, D, MODEL>(Q, Jb, ph, P, Sv, dl);
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] += Q[k];
    acc[K] += dl;
    acc[K + 1] += dl * dl;
    acc[K + 2] = fmax(acc[K + 2], fabs(dl));
    acc[K + 4] += bad ? 1.0 : 0.0;
  }
  block_reduce<NT>(acc, NT, 1u << (K + 2), partial + (size_t)blockIdx.x * NT);
}

// Network input of the learned correction (8-variable ideal model): the moments of
// each cell in the storage's compute type, summed over i in order, then as FP32 and
// standardised BF16 (round to nearest even), one cell per thread.
template <int ST, int D>
__global__ __launch_bounds__(256) void k_net_input(const Grid g, const Codec cd, int parity, const MomentsOut mo) {
  using S = Store<ST>;
  using T = typename S::T;
  using R = typename S::R;
  constexpr int NQ = 2 * D + 1, K = 8;
  const T* __restrict__ F = static_cast<const T*>(g.f);
  const size_t N = (size_t)g.nx * g.ny * g.nz;
  const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  const int x = (int)(c % g.nx), y = (int)((c / g.nx) % g.ny), z = (int)(c / ((size_t)g.nx * g.ny));
  unsigned np[3], nm[3];
  neighbours<D>(g, x, y, z, (unsigned)c, np, nm);
  unsigned h[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    R q = R(0);
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      const unsigned src = (parity == 0 || i == 0) ? (unsigned)c : ((i & 1) ? nm[(i - 1) >> 1] : np[(i - 1) >> 1]);
      const int slot = parity == 0 ? i : opposite(i);
      q += S::dec(F[(size_t)(k * NQ + slot) * g.stride + src], cd, k * NQ + i);
    }
    const float xq = (float)q;
    mo.x[(size_t)k * N + c] = xq;
    const unsigned u = __float_as_uint((xq - mo.mean[k]) * mo.istd[k]);
    h[k] = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
  }
  *reinterpret_cast<uint4*>(mo.act + c * K) =
      make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16));
}

// Per-step loads on the homogenized body at time b.t (cells of b.box): what the
// homogenized collision moves from the fluid to the body -- force (momentum), torque
// about the body's centre, energy -- and the magnetic flux through its surface,
// 1/2 sum |B . r/|r|| over the one-cell porosity ramp.  The cell's moments change by
// omega_k (Q^_k - Q_k) in the collision; omega_k = 1/tau_k (BGK), the symmetric rate
// (two-rate collisions carry the zeroth moment in the symmetric halves), 1 (RLB).
// partial[block][8] = (F, T, W, flux).
template <int ST>
__global__ __launch_bounds__(kReduceThreads) void k_body_loads(const Grid g, const Phys ph, const Codec cd,
                                                               int parity, const Body b,
                                                               double* __restrict__ partial) {
  using R = typename Store<ST>::R;
  double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const long long bx = b.box[1] - b.box[0], by = b.box[3] - b.box[2], bz = b.box[5] - b.box[4];
  const long long nb = bx * by * bz;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < nb; t += (long long)gridDim.x * blockDim.x) {
    const int x = b.box[0] + (int)(t % bx), y = b.box[2] + (int)((t / bx) % by), z = b.box[4] + (int)(t / (bx * by));
    const HlbmTarget tg{&b, x, y, z, HlbmTarget::near_body(b, x, y, z), ph.s, ph.gm1};
    if (!tg.near) continue;
    double r[3], rr;
    const double phi = tg.rr_minus_R(r, rr);
    if (phi >= 0.5) continue;  // porosity 1: fluid, no exchange
    const unsigned c = (unsigned)x + (unsigned)g.nx * ((unsigned)y + (unsigned)g.ny * (unsigned)z);
    R Qr[8];
    cell_moments3<ST>(g, cd, parity, c, Qr);
    double Q[8], Qh[8];
    for (int k = 0; k < 8; ++k) Q[k] = Qh[k] = (double)Qr[k];
    tg(Qh);
    double om[5];
    for (int k = 1; k < 5; ++k) om[k] = ph.collision == 0 ? ph.omega[k] : (ph.collision == 1 ? ph.omega_s[k] : 1.0);
    const double dM[3] = {om[1] * (Qh[1] - Q[1]), om[2] * (Qh[2] - Q[2]), om[3] * (Qh[3] - Q[3])};
    acc[0] -= dM[0];
    acc[1] -= dM[1];
    acc[2] -= dM[2];
    acc[3] -= r[1] * dM[2] - r[2] * dM[1];
    acc[4] -= r[2] * dM[0] - r[0] * dM[2];
    acc[5] -= r[0] * dM[1] - r[1] * dM[0];
    acc[6] -= om[4] * (Qh[4] - Q[4]);
    if (phi > -0.5 && rr > 0.0) acc[7] += 0.5 * fabs(Q[5] * r[0] + Q[6] * r[1] + Q[7] * r[2]) / rr;
  }
  block_reduce<8>(acc, 8, 0u, partial + (size_t)blockIdx.x * 8);
}

// bx: index of B_x in the moment field
template <int D>
__global__ __launch_bounds__(kReduceThreads) void k_divc(const Grid g, const double* __restrict__ Qm, int bx,
                                                         double* __restrict__ partial) {
  const size_t N = (size_t)g.nx * g.ny * g.nz;
  double acc[1] = {0.0};
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < N;
       c += (size_t)gridDim.x * blockDim.x) {
    const int x = (int)(c % g.nx);
    const int y = (int)((c / g.nx) % g.ny);
    const int z = (int)(c / ((size_t)g.nx * g.ny));
    unsigned np[3], nm[3];
    neighbours<D>(g, x, y, z, (unsigned)c, np, nm);
    double dv = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) dv += 0.5 * (Qm[(size_t)(bx + a) * N + np[a]] - Qm[(size_t)(bx + a) * N + nm[a]]);
    acc[0] += dv * dv;
  }
  block_reduce<1>(acc, 1, 0u, partial + blockIdx.x);
}

template <int NMAX>
__global__ __launch_bounds__(kReduceThreads) void k_reduce(int n, const double* __restrict__ partial,
                                                           int nblk, unsigned maxmask,
                                                           double* __restrict__ out) {
  double acc[NMAX];
#pragma unroll
  for (int j = 0; j < NMAX; ++j) acc[j] = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x)
    for (int j = 0; j < n; ++j) {
      const double v = partial[(size_t)b * n + j];
      acc[j] = ((maxmask >> j) & 1u) ? fmax(acc[j], v) : acc[j] + v;
    }
  block_reduce<NMAX>(acc, n, maxmask, out);
}

// per-variable sum (mode 0) or max |Q_k - rest_k| (mode 1) over the field
template <int NMAX, typename QT>
__global__ __launch_bounds__(kReduceThreads) void k_field_reduce(const QT* __restrict__ Q, long long N,
                                                                 int K, int mode,
                                                                 const double* __restrict__ rest,
                                                                 double* __restrict__ partial) {
  double acc[NMAX];
#pragma unroll
  for (int j = 0; j < NMAX; ++j) acc[j] = 0.0;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < N;
       c += (long long)gridDim.x * blockDim.x)
    for (int k = 0; k < K; ++k) {
      const double v = (double)Q[(size_t)k * N + c];
      acc[k] = mode == 0 ? acc[k] + v : fmax(acc[k], fabs(v - rest[k]));
    }
  block_reduce<NMAX>(acc, K, mode == 0 ? 0u : 0xffffffffu, partial + (size_t)blockIdx.x * K);
}

template <int ST, int D>
__global__ void k_gather(const Grid g, const Codec cd, int parity, int K,
                         const long long* __restrict__ cells, long long n, double* __restrict__ out) {
  using S = Store<ST>;
  using T = typename S::T;
  constexpr int NQ = 2 * D + 1;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * K * NQ) return;
  const int i = (int)(t % NQ);
  const int k = (int)((t / NQ) % K);
  const long long c = cells[t / ((long long)NQ * K)];
  const int x = (int)(c % g.nx);
  const int y = (int)((c / g.nx) % g.ny);
  const int z = (int)(c / ((long long)g.nx * g.ny));
  unsigned np[3], nm[3];
  neighbours<D>(g, x, y, z, (unsigned)c, np, nm);
  const unsigned src = (parity == 0 || i == 0) ? (unsigned)c : ((i & 1) ? nm[(i - 1) >> 1] : np[(i - 1) >> 1]);
  const int slot = parity == 0 ? i : opposite(i);
  const T* F = static_cast<const T*>(g.f);
  out[t] = S::dec64(F[pop_index(g, NQ, k, slot, src)], cd, k * NQ + i);
}

__global__ void k_to_f32(const double* __restrict__ in, float* __restrict__ out, long long n) {
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (long long)gridDim.x * blockDim.x)
    out[t] = (float)in[t];
}

// One 16-byte element per thread and no grid-stride loop: the fastest plain copy
// form measured on gfx950 (a grid-stride loop over 8192 blocks reaches ~77 % of it).
__global__ __launch_bounds__(256) void k_copy(uint4* __restrict__ dst, const uint4* __restrict__ src,
                                              size_t n) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) dst[t] = src[t];
}

// ---------------------------------------------------------------------------
// launch helpers
// ---------------------------------------------------------------------------

template <int ST>
hipError_t boundary_t(const Launch& L, const Grid& g, const Phys& ph, const Codec& cd, int parity,
                      const Body* b, const Inflow* in, int what) {
  if (what == 0) {  // faces
    const long long area = std::max({(long long)g.ny * g.nz, (long long)g.nx * g.nz, (long long)g.nx * g.ny});
    hipLaunchKernelGGL((k_faces<ST>), dim3((unsigned)((area + 255) / 256), 1, 6), dim3(256), 0, L.stream, g, ph,
                       cd, parity, *in);
  } else {  // refill
    const long long n = (long long)(b->box[1] - b->box[0]) * (b->box[3] - b->box[2]) * (b->box[5] - b->box[4]);
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_refill<ST>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, L.stream, g, ph, cd,
                       parity, *b, *in);
  }
  return hipGetLastError();
}

hipError_t boundary(const Launch& L, const Grid& g, const Phys& ph, const Codec& cd, int parity, const Body* b,
                    const Inflow* in, int what) {
  if (L.dim != 3 || L.model != 0) return hipErrorInvalidValue;
  switch (L.storage) {
    case ST_F64: return boundary_t<ST_F64>(L, g, ph, cd, parity, b, in, what);
    case ST_F32: return boundary_t<ST_F32>(L, g, ph, cd, parity, b, in, what);
    case ST_F16: return boundary_t<ST_F16>(L, g, ph, cd, parity, b, in, what);
    case ST_BF16: return boundary_t<ST_BF16>(L, g, ph, cd, parity, b, in, what);
    default: return hipErrorInvalidValue;
  }
}

template <int ST, int D, int MODEL>
hipError_t init_t(const Launch& L, const Grid& g, const Phys& ph, const Codec& cd, const void* Q,
                  int f32) {
  const dim3 grd = cell_grid(g, L.block_x), blk(L.block_x);
  if (f32)
    hipLaunchKernelGGL((k_init<ST, D, MODEL, float>), grd, blk, 0, L.stream, g, ph, cd,
                       static_cast<const float*>(Q));
  else
    hipLaunchKernelGGL((k_init<ST, D, MODEL, double>), grd, blk, 0, L.stream, g, ph, cd,
                       static_cast<const double*>(Q));
  return hipGetLastError();
}

template <int ST, int D, int MODEL>
hipError_t moments_t(const Launch& L, const Grid& g, const Phys& ph, const Codec& cd, int parity,
                     double* Qout, double* partial, int nblk) {
  hipLaunchKernelGGL((k_moments<ST, D, MODEL>), dim3(nblk), dim3(kReduceThreads), 0, L.stream, g,
                     ph, cd, parity, Qout, partial);
  return hipGetLastError();
}

template <int ST>
hipError_t gather_t(const Launch& L, const Grid& g, const Codec& cd, int parity, int K,
                    const long long* cells, long long n, double* out) {
  const long long tot = n * K * (2 * L.dim + 1);
  const dim3 grd((unsigned)((tot + 255) / 256)), blk(256);
  if (L.dim == 2)
    hipLaunchKernelGGL((k_gather<ST, 2>), grd, blk, 0, L.stream, g, cd, parity, K, cells, n, out);
  else
    hipLaunchKernelGGL((k_gather<ST, 3>), grd, blk, 0, L.stream, g, cd, parity, K, cells, n, out);
  return hipGetLastError();
}

template <int ST, int D, int M>
struct InitFn {
  static hipError_t run(const Launch& L, const Grid& g, const Phys& ph, const Codec& cd,
                        const void* Q, int f32) {
    return init_t<ST, D, M>(L, g, ph, cd, Q, f32);
  }
};
template <int ST, int D, int M>
struct MomentsFn {
  static hipError_t run(const Launch& L, const Grid& g, const Phys& ph, const Codec& cd, int par,
                        double* Qout, double* partial, int nblk) {
    return moments_t<ST, D, M>(L, g, ph, cd, par, Qout, partial, nblk);
  }
};

}  // namespace

hipError_t launch_net_input(const Launch& L, const Grid& g, const Codec& cd, int parity, const MomentsOut& mo) {
  const size_t N = (size_t)g.nx * g.ny * g.nz;
  const dim3 grd((unsigned)((N + 255) / 256)), blk(256);
  switch (L.storage * 2 + (L.dim - 2)) {
#define NI_CASE(ST, D)                                                                               \
  case ST * 2 + (D - 2):                                                                             \
    hipLaunchKernelGGL((k_net_input<ST, D>), grd, blk, 0, L.stream, g, cd, parity, mo);              \
    return hipGetLastError();
    NI_CASE(ST_F64, 2) NI_CASE(ST_F64, 3) NI_CASE(ST_F32, 2) NI_CASE(ST_F32, 3)
    NI_CASE(ST_F16, 2) NI_CASE(ST_F16, 3) NI_CASE(ST_BF16, 2) NI_CASE(ST_BF16, 3)
#undef NI_CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_init(const Launch& L, const Grid& g, const Phys& ph, const Codec& cd,
                       const void* Q, int q_is_f32) {
  return dispatch<InitFn>(L, g, ph, cd, Q, q_is_f32);
}

hipError_t launch_faces(const Launch& L, const Grid& g, const Phys& ph, const Codec& cd, int parity,
                        const Inflow& in) {
  return boundary(L, g, ph, cd, parity, nullptr, &in, 0);
}

hipError_t launch_refill(const Launch& L, const Grid& g, const Phys& ph, const Codec& cd, int parity,
                         const Body& b, const Inflow& in) {
  if (!g.mask) return hipErrorInvalidValue;
  return boundary(L, g, ph, cd, parity, &b, &in, 2);
}

hipError_t launch_mask(const Launch& L, const Grid& g, const Body& b, int pass, int fresh) {
  if (!g.mask) return hipErrorInvalidValue;
  const long long n = (long long)(b.box[1] - b.box[0]) * (b.box[3] - b.box[2]) * (b.box[5] - b.box[4]);
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mask, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, L.stream, g, b, pass, fresh);
  return hipGetLastError();
}

hipError_t launch_moments(const Launch& L, const Grid& g, const Phys& ph, const Codec& cd,
                          int parity, double* Qout, double* partial, int nblk) {
  return dispatch<MomentsFn>(L, g, ph, cd, parity, Qout, partial, nblk);
}

hipError_t launch_divc(const Launch& L, const Grid& g, const double* Qout, double* partial, int nblk) {
  const int bx = L.model == 4 ? kBx<4> : kBx<0>;
  if (L.dim == 2)
    hipLaunchKernelGGL((k_divc<2>), dim3(nblk), dim3(kReduceThreads), 0, L.stream, g, Qout, bx, partial);
  else
    hipLaunchKernelGGL((k_divc<3>), dim3(nblk), dim3(kReduceThreads), 0, L.stream, g, Qout, bx, partial);
  return hipGetLastError();
}

hipError_t launch_body_loads(const Launch& L, const Grid& g, const Phys& ph, const Codec& cd, int parity,
                             const Body& b, double* partial, int nblk) {
  if (L.dim != 3 || L.model != 0) return hipErrorInvalidValue;
  const dim3 grd(nblk), blk(kReduceThreads);
  switch (L.storage) {
    case ST_F64: hipLaunchKernelGGL(k_body_loads<ST_F64>, grd, blk, 0, L.stream, g, ph, cd, parity, b, partial); break;
    case ST_F32: hipLaunchKernelGGL(k_body_loads<ST_F32>, grd, blk, 0, L.stream, g, ph, cd, parity, b, partial); break;
    case ST_F16: hipLaunchKernelGGL(k_body_loads<ST_F16>, grd, blk, 0, L.stream, g, ph, cd, parity, b, partial); break;
    case ST_BF16: hipLaunchKernelGGL(k_body_loads<ST_BF16>, grd, blk, 0, L.stream, g, ph, cd, parity, b, partial); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_reduce(const Launch& L, int n, const double* partial, int nblk, unsigned maxmask,
                         double* out) {
  if (n > 32) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_reduce<32>), dim3(1), dim3(kReduceThreads), 0, L.stream, n, partial, nblk,
                     maxmask, out);
  return hipGetLastError();
}

hipError_t launch_gather(const Launch& L, const Grid& g, const Codec& cd, int parity, int K,
                         const long long* cells, long long n, double* out) {
  switch (L.storage) {
    case ST_F64: return gather_t<ST_F64>(L, g, cd, parity, K, cells, n, out);
    case ST_F32: return gather_t<ST_F32>(L, g, cd, parity, K, cells, n, out);
    case ST_F16: return gather_t<ST_F16>(L, g, cd, parity, K, cells, n, out);
    case ST_BF16: return gather_t<ST_BF16>(L, g, cd, parity, K, cells, n, out);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_field_reduce(const Launch& L, long long N, int K, const void* Q, int q_is_f32,
                               int mode, const double* rest, double* partial, int nblk, double* out) {
  if (K > 32) return hipErrorInvalidValue;
  if (q_is_f32)
    hipLaunchKernelGGL((k_field_reduce<32, float>), dim3(nblk), dim3(kReduceThreads), 0, L.stream,
                       static_cast<const float*>(Q), N, K, mode, rest, partial);
  else
    hipLaunchKernelGGL((k_field_reduce<32, double>), dim3(nblk), dim3(kReduceThreads), 0, L.stream,
                       static_cast<const double*>(Q), N, K, mode, rest, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_reduce(L, K, partial, nblk, mode == 0 ? 0u : 0xffffffffu, out);
}

hipError_t launch_to_f32(hipStream_t s, const double* in, float* out, long long n) {
  hipLaunchKernelGGL(k_to_f32, dim3(1024), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}

hipError_t launch_copy(hipStream_t s, void* dst, const void* src, size_t bytes) {
  const size_t n = bytes / 16;
  const size_t blocks = (n + 255) / 256;
  if (blocks == 0) return hipSuccess;
  if (blocks > 0x7fffffffULL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<uint4*>(dst),
                     static_cast<const uint4*>(src), n);
  return hipGetLastError();
}

}  // namespace vlbm

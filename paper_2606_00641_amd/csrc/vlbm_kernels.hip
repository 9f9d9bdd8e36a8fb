// HIP kernels (gfx950) of the VLBM MHD sweep and its diagnostics.
//
// Data layout in HBM: one population buffer, SoA planes indexed (k*Q + i) of
// `stride` elements, cell index c = x + nx (y + ny z) with x fastest, so a
// wavefront touches 64 consecutive cells of one plane per access.
//
// Streaming is the in-place AA pattern: a step at parity 0 reads slot i of its
// own cell and writes the post-collision value of direction i to slot opposite(i)
// of the same cell; a step at parity 1 reads slot opposite(i) of cell x - e_i and
// writes slot i of cell x + e_i.  Every slot is read and written by one thread
// only, so one buffer suffices and there is no race.  After a parity-0 step the
// pre-collision population f_i(x) sits at slot opposite(i) of cell x - e_i; after
// a parity-1 step the layout is natural again.
#include <algorithm>

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "vlbm_kernels.h"

namespace vlbm {
namespace {

constexpr int kReduceThreads = 256;

// ---------------------------------------------------------------------------
// storage codecs
// ---------------------------------------------------------------------------
template <int ST>
struct Store;

template <>
struct Store<ST_F64> {
  using T = double;
  using R = double;
  static __device__ __forceinline__ R dec(T v, const Codec&, int) { return v; }
  static __device__ __forceinline__ T enc(R v, const Codec&, int) { return v; }
  static __device__ __forceinline__ double dec64(T v, const Codec&, int) { return v; }
};

template <>
struct Store<ST_F32> {
  using T = float;
  using R = float;
  static __device__ __forceinline__ R dec(T v, const Codec&, int) { return v; }
  static __device__ __forceinline__ T enc(R v, const Codec&, int) { return v; }
  static __device__ __forceinline__ double dec64(T v, const Codec&, int) { return v; }
};

template <>
struct Store<ST_F16> {
  using T = unsigned short;
  using R = float;
  static __device__ __forceinline__ float h2f(T v) { return __half2float(__ushort_as_half(v)); }
  static __device__ __forceinline__ R dec(T v, const Codec& cd, int j) {
    return fmaf(cd.sc[j], h2f(v), cd.rest[j]);
  }
  static __device__ __forceinline__ T enc(R v, const Codec& cd, int j) {
    float h = (v - cd.rest[j]) * cd.isc[j];
    h = fminf(fmaxf(h, -65504.0f), 65504.0f);  // saturate instead of overflowing to inf
    return __half_as_ushort(__float2half_rn(h));
  }
  static __device__ __forceinline__ double dec64(T v, const Codec& cd, int j) {
    return (double)cd.rest[j] + (double)cd.sc[j] * (double)h2f(v);
  }
};

template <>
struct Store<ST_BF16> {
  using T = unsigned short;
  using R = float;
  static __device__ __forceinline__ float b2f(T v) { return __uint_as_float((unsigned)v << 16); }
  static __device__ __forceinline__ R dec(T v, const Codec& cd, int j) {
    return fmaf(cd.sc[j], b2f(v), cd.rest[j]);
  }
  static __device__ __forceinline__ T enc(R v, const Codec& cd, int j) {
    const float h = (v - cd.rest[j]) * cd.isc[j];
    // round to nearest even on the upper 16 bits (finite inputs)
    const unsigned u = __float_as_uint(h);
    return (T)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
  }
  static __device__ __forceinline__ double dec64(T v, const Codec& cd, int j) {
    return (double)cd.rest[j] + (double)cd.sc[j] * (double)b2f(v);
  }
};

// Neighbour linear indices of cell (x, y, z) along +e_a (np) and -e_a (nm),
// periodic.  32-bit: every supported lattice has fewer than 2^31 cells.
template <int D>
__device__ __forceinline__ void neighbours(const Grid& g, int x, int y, int z, unsigned c,
                                           unsigned (&np)[3], unsigned (&nm)[3]) {
  const unsigned nx = g.nx, pl = (unsigned)g.nx * (unsigned)g.ny;
  np[0] = (x + 1 == g.nx) ? c + 1 - nx : c + 1;
  nm[0] = (x == 0) ? c + nx - 1 : c - 1;
  np[1] = (y + 1 == g.ny) ? c - (unsigned)(g.ny - 1) * nx : c + nx;
  nm[1] = (y == 0) ? c + (unsigned)(g.ny - 1) * nx : c - nx;
  if constexpr (D == 3) {
    np[2] = (z + 1 == g.nz) ? c - (unsigned)(g.nz - 1) * pl : c + pl;
    nm[2] = (z == 0) ? c + (unsigned)(g.nz - 1) * pl : c - pl;
  } else {
    np[2] = nm[2] = c;
  }
}

// ---------------------------------------------------------------------------
// the sweep: gather, decode, collide (moments, EOS, fluxes, div B, Powell, BGK +
// injection), encode, scatter
// ---------------------------------------------------------------------------
// Plane addressing: the base of plane (k*Q + i) is wavefront-uniform, the per-lane
// part is a 32-bit byte offset, so loads and stores use the scalar-base +
// vector-offset form and keep no 64-bit address per population in registers.
// (The library rejects lattices whose plane exceeds 4 GiB.)
#define VLBM_GLOBAL __attribute__((address_space(1)))

__device__ __forceinline__ VLBM_GLOBAL char* plane_base(void* base, size_t plane_bytes, int plane) {
  // The base is the same for every lane; reading it through readfirstlane keeps it
  // an opaque scalar value, so the backend cannot first fold the lane offset into
  // it (which would cost a 64-bit VGPR address per load), and the global address
  // space lets it use the scalar-base form of the load.
  const unsigned long long a = reinterpret_cast<unsigned long long>(base) + plane_bytes * plane;
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)a);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(a >> 32));
  return (VLBM_GLOBAL char*)(((unsigned long long)hi << 32) | lo);
}
// Loads and stores are nontemporal: every population is read once and written once
// per sweep, and keeping the streams out of the caches measurably raised the sweep's
// bandwidth on gfx950 (stores: +3 %; loads, on top: +4 % on the 26-variable FP32
// sweep, +7 % FP32 / +14 % FP16 on the 8-variable sweep).
template <typename T>
__device__ __forceinline__ T ld(void* base, size_t plane_bytes, int plane, unsigned off) {
  return __builtin_nontemporal_load((const VLBM_GLOBAL T*)(plane_base(base, plane_bytes, plane) + off));
}
template <typename T>
__device__ __forceinline__ void st(void* base, size_t plane_bytes, int plane, unsigned off, T v) {
  __builtin_nontemporal_store(v, (VLBM_GLOBAL T*)(plane_base(base, plane_bytes, plane) + off));
}

// Dipole field of the body at point q (cell coordinates) and time t.
__device__ inline void dipole_at(const Body& b, const double (&q)[3], double t, double (&B)[3]) {
  double r[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) r[a] = q[a] - (b.c0[a] + t * b.v[a]);
  const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
  const double r5 = r2 * r2 * sqrt(r2);
  const double mr = b.m[0] * r[0] + b.m[1] * r[1] + b.m[2] * r[2];
#pragma unroll
  for (int a = 0; a < 3; ++a) B[a] = (3.0 * mr * r[a] - b.m[a] * r2) / r5;
}

// Solid test of the rough sphere: the cell centre lies strictly inside the surface
// radius R0 (1 + delta(direction)), delta a sum of dipolar (d_j . n) and quadrupolar
// ((e_j . n)^2 - 1/3) terms.  Evaluated in FP64 without contraction, operation by
// operation, so that every cell gets the same decision as a plain IEEE evaluation.
__device__ inline double surface_radius(const Body& b, int x, int y, int z, double t, double (&r)[3],
                                        double& rr) {
#pragma clang fp contract(off)
  r[0] = x - (b.c0[0] + t * b.v[0]);
  r[1] = y - (b.c0[1] + t * b.v[1]);
  r[2] = z - (b.c0[2] + t * b.v[2]);
  rr = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  if (rr == 0.0) return b.R0;
  double delta = 0.0;
  for (int j = 0; j < 4; ++j) {
    double dn = 0.0, en = 0.0;
    for (int a = 0; a < 3; ++a) {
      dn += b.d[j][a] * r[a] / rr;
      en += b.e[j][a] * r[a] / rr;
    }
    delta += b.a[j] * dn + b.b[j] * (en * en - 1.0 / 3.0);
  }
  return b.R0 * (1.0 + delta);
}

__device__ inline bool body_solid(const Body& b, int x, int y, int z, double t) {
  double r[3], rr;
  const double R = surface_radius(b, x, y, z, t, r, rr);
  return rr == 0.0 || rr < R;
}

// Homogenized collision target (Sec. 2.4): porosity d from the radial signed
// distance phi = |r| - R(n) with a linear transition one cell wide; u and B are
// blended with the body's velocity (v / s in flux units) and field (dipole outside
// R0, the uniform 2 m / R0^3 of a magnetised sphere inside); rho and the pressure
// are kept and e_tot follows.  Cells beyond the surface-radius bound are fluid
// (d = 1) and skip the geometry.
struct HlbmTarget {
  const Body* b;
  int x, y, z;
  bool near;  // within the surface-radius bound plus half a cell
  double s, gm1;
  static __device__ __forceinline__ bool near_body(const Body& b, int x, int y, int z) {
    const double t = b.t;
    const double cx = x - (b.c0[0] + t * b.v[0]), cy = y - (b.c0[1] + t * b.v[1]),
                 cz = z - (b.c0[2] + t * b.v[2]);
    const double lim = b.rmax + 0.5;
    return cx * cx + cy * cy + cz * cz < lim * lim;
  }
  template <typename R>
  __device__ __forceinline__ void operator()(R* Q) const {
    if (!near) return;
    double r[3], rr;
    const double phi = rr_minus_R(r, rr);
    double d;
    if (phi <= -0.5)
      d = 0.0;
    else if (phi >= 0.5)
      return;
    else
      d = phi + 0.5;
    const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    double Bb[3];
    if (r2 < b->R0 * b->R0) {
      for (int a = 0; a < 3; ++a) Bb[a] = 2.0 * b->m[a] / (b->R0 * b->R0 * b->R0);
    } else {
      const double r5 = r2 * r2 * sqrt(r2);
      const double mr = b->m[0] * r[0] + b->m[1] * r[1] + b->m[2] * r[2];
      for (int a = 0; a < 3; ++a) Bb[a] = (3.0 * mr * r[a] - b->m[a] * r2) / r5;
    }
    const R rho = Q[0], dd = R(d), ed = R(1.0 - d), g1 = R(gm1);
    const R ir = R(1) / rho;
    R uu = R(0), BB = R(0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const R u = Q[1 + a] * ir;
      uu += u * u;
      BB += Q[5 + a] * Q[5 + a];
    }
    const R pres = g1 * (Q[4] - R(0.5) * rho * uu - R(0.5) * BB);
    R uh2 = R(0), Bh2 = R(0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const R uh = dd * (Q[1 + a] * ir) + ed * R(b->v[a] / s);
      const R Bh = dd * Q[5 + a] + ed * R(Bb[a]);
      Q[1 + a] = rho * uh;
      Q[5 + a] = Bh;
      uh2 += uh * uh;
      Bh2 += Bh * Bh;
    }
    Q[4] = pres / g1 + R(0.5) * rho * uh2 + R(0.5) * Bh2;
  }
  __device__ double rr_minus_R(double (&r)[3], double& rr) const {
    const double R = surface_radius(*b, x, y, z, b->t, r, rr);
    return rr - R;
  }
};

// BODY (D3Q7 ideal): solid cells are skipped; a link i whose neighbour x + e_i is
// solid returns the post-collision population into direction opposite(i) of the
// same cell -- halfway bounce-back with the moving-wall flux correction for rho and
// E, anti-bounce-back to rho u_w and to the dipole field at the link midpoint for
// rho u and B.  In the AA layout that population belongs at slot i of cell x + e_i
// after a parity-0 step and at slot opposite(i) of x after a parity-1 step, places
// no other thread writes because the solid cell runs no update.
// INJ: before the collision add *dqflag * w_i dq[k][c] to f_{k,i} (the pending learned
// coarse correction, which shifts the zeroth moments by dq); dq is FP32 [K][N].
template <int ST, int D, int MODEL, int PAR, int BODY = 0, int COLL = 0, bool INJ = false>
__global__ __launch_bounds__(256) void k_sweep(const Grid g, const Phys ph, const Codec cd,
                                               const Body bd = Body{}, const float* __restrict__ dq = nullptr,
                                               const int* __restrict__ dqflag = nullptr) {
  using S = Store<ST>;
  using T = typename S::T;
  using R = typename S::R;
  constexpr int NQ = 2 * D + 1;
  constexpr int K = MODEL ? 26 : 8;
  constexpr unsigned ES = sizeof(T);
  // BODY 2 runs over the body's box only (grid = box extent, offset by its corner);
  // BODY 3 is the plain sweep of every other cell.
  int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
  if constexpr (BODY == 2) {
    x += bd.box[0];
    y += bd.box[2];
    z += bd.box[4];
    if (x >= bd.box[1]) return;
  } else {
    if (x >= g.nx) return;
  }
  if constexpr (BODY == 3) {
    if (x >= bd.box[0] && x < bd.box[1] && y >= bd.box[2] && y < bd.box[3] && z >= bd.box[4] && z < bd.box[5])
      return;
  }
  const unsigned c = (unsigned)x + (unsigned)g.nx * ((unsigned)y + (unsigned)g.ny * (unsigned)z);
  void* const F = g.f;
  const size_t pb = (size_t)g.stride * ES;
  unsigned mk = 0;
  if constexpr (BODY == 1) {
    mk = g.mask[c];
    if (mk & kSolid) return;
  }

  // byte offsets of this cell and of its neighbours x + e_a (np), x - e_a (nm)
  unsigned np[3], nm[3];
  if constexpr (PAR == 1 || BODY == 1) {
    neighbours<D>(g, x, y, z, c, np, nm);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      np[a] *= ES;
      nm[a] *= ES;
    }
  }
  const unsigned co = c * ES;

  R f[K][NQ];
#pragma unroll
  for (int k = 0; k < K; ++k) {
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      T v;
      if constexpr (PAR == 0) {
        v = ld<T>(F, pb, k * NQ + i, co);
      } else {
        // f_i(x) was written by cell x - e_i into its slot opposite(i)
        const unsigned src = (i == 0) ? co : ((i & 1) ? nm[(i - 1) >> 1] : np[(i - 1) >> 1]);
        v = ld<T>(F, pb, k * NQ + opposite(i), src);
      }
      f[k][i] = S::dec(v, cd, k * NQ + i);
    }
  }

  if constexpr (INJ) {
    if (*dqflag) {
      const size_t N = (size_t)g.nx * g.ny * g.nz;
      const R wi = R(ph.wi);
      const R w0 = rest_weight<R, D>(wi);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const R d = (R)dq[(size_t)k * N + c];
#pragma unroll
        for (int i = 0; i < NQ; ++i) f[k][i] += (i == 0 ? w0 : wi) * d;
      }
    }
  }

  R dl;
  if constexpr (BODY != 1) {
    if constexpr (BODY == 2) {
      static_assert(D == 3 && MODEL == 0, "homogenized body: D3Q7 ideal MHD");
      R Q[K], pt;
      const bool near = HlbmTarget::near_body(bd, x, y, z);
      collide<R, D, MODEL, COLL>(f, ph, dl, Q, pt, HlbmTarget{&bd, x, y, z, near, ph.s, ph.gm1});
    } else {
      collide<R, D, MODEL, COLL>(f, ph, dl);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
#pragma unroll
      for (int i = 0; i < NQ; ++i) {
        const T v = S::enc(f[k][i], cd, k * NQ + i);
        if constexpr (PAR == 0) {
          st<T>(F, pb, k * NQ + opposite(i), co, v);
        } else {
          const unsigned dst = (i == 0) ? co : ((i & 1) ? np[(i - 1) >> 1] : nm[(i - 1) >> 1]);
          st<T>(F, pb, k * NQ + i, dst, v);
        }
      }
    }
  } else {
    static_assert(D == 3 && MODEL == 0, "body bounce-back: D3Q7 ideal MHD");
    R Q[K], pt;
    collide<R, D, MODEL, COLL>(f, ph, dl, Q, pt);
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      const unsigned dst = (i == 0) ? co : ((i & 1) ? np[(i - 1) >> 1] : nm[(i - 1) >> 1]);
      if (i > 0 && (mk & link_bit(i))) {
        const int a = (i - 1) >> 1;
        const R sg = (i & 1) ? R(1) : R(-1);
        const double q[3] = {x + (a == 0 ? 0.5 * (double)sg : 0.0), y + (a == 1 ? 0.5 * (double)sg : 0.0),
                             z + (a == 2 ? 0.5 * (double)sg : 0.0)};
        double Bw[3];
        dipole_at(bd, q, bd.t, Bw);
        // wall velocity in flux units: v cells per step is the velocity v / s
        const R uw[3] = {R(bd.v[0] / ph.s), R(bd.v[1] / ph.s), R(bd.v[2] / ph.s)};
        const R rho = Q[0], E = Q[4];
        const R uB = uw[0] * Q[5] + uw[1] * Q[6] + uw[2] * Q[7];
        const R c = R(2.0 * ph.wi * ph.inv_cs2 * ph.s) * sg;
        const R w2 = R(2.0 * ph.wi);
        R out[K];
        out[0] = f[0][i] - c * rho * uw[a];
        out[4] = f[4][i] - c * ((E + pt) * uw[a] - Q[5 + a] * uB);
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          out[1 + b] = -f[1 + b][i] + w2 * rho * uw[b];
          out[5 + b] = -f[5 + b][i] + w2 * R(Bw[b]);
        }
        const int ib = opposite(i);
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const T v = S::enc(out[k], cd, k * NQ + ib);
          if constexpr (PAR == 0)
            st<T>(F, pb, k * NQ + i, dst, v);
          else
            st<T>(F, pb, k * NQ + ib, co, v);
        }
      } else {
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const T v = S::enc(f[k][i], cd, k * NQ + i);
          if constexpr (PAR == 0)
            st<T>(F, pb, k * NQ + opposite(i), co, v);
          else
            st<T>(F, pb, k * NQ + i, dst, v);
        }
      }
    }
  }
}

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
// on several non-periodic faces is handled by each of them with identical values;
// the cells read (no non-periodic face) and the populations written (face nodes
// only) are disjoint.
template <int ST>
__global__ __launch_bounds__(256) void k_faces(const Grid g, const Phys ph, const Codec cd, int parity,
                                               const Inflow in) {
  using R = typename Store<ST>::R;
  const int f = blockIdx.z, a = f >> 1;
  if (g.bc[f] == 0) return;
  const int n[3] = {g.nx, g.ny, g.nz};
  const int a1 = (a + 1) % 3, a2 = (a + 2) % 3;
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
  constexpr int K = MODEL ? 26 : 8;
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
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int i = 0; i < NQ; ++i)
      F[(size_t)(k * NQ + i) * g.stride + c] = S::enc(feq_dir<R, D>(Q[k], P[k], i, w0, wi), cd, k * NQ + i);
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
  constexpr int K = MODEL ? 26 : 8;
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
        const double v = S::dec64(F[(size_t)(k * NQ + slot) * g.stride + src], cd, k * NQ + i);
        q += v;
        if (k >= 5 && k < 5 + D && i > 0 && ((i - 1) >> 1) == k - 5) Jb[k - 5] += (i & 1) ? v : -v;
      }
      Q[k] = q;
      Qout[(size_t)k * N + c] = q;
    }
    double P[K][3], Sv[K], dl;
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

template <int D>
__global__ __launch_bounds__(kReduceThreads) void k_divc(const Grid g, const double* __restrict__ Qm,
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
    for (int a = 0; a < D; ++a) dv += 0.5 * (Qm[(size_t)(5 + a) * N + np[a]] - Qm[(size_t)(5 + a) * N + nm[a]]);
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
  out[t] = S::dec64(F[(size_t)(k * NQ + slot) * g.stride + src], cd, k * NQ + i);
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
dim3 cell_grid(const Grid& g, int bx) { return dim3((g.nx + bx - 1) / bx, g.ny, g.nz); }

template <int ST, int D, int MODEL>
hipError_t sweep_t(const Launch& L, const Grid& g, const Phys& ph, const Codec& cd, int parity) {
  const dim3 grd = cell_grid(g, L.block_x), blk(L.block_x);
  switch ((ph.collision ? 2 : 0) + parity) {
    case 0: hipLaunchKernelGGL((k_sweep<ST, D, MODEL, 0, 0, 0>), grd, blk, 0, L.stream, g, ph, cd); break;
    case 1: hipLaunchKernelGGL((k_sweep<ST, D, MODEL, 1, 0, 0>), grd, blk, 0, L.stream, g, ph, cd); break;
    case 2: hipLaunchKernelGGL((k_sweep<ST, D, MODEL, 0, 0, 1>), grd, blk, 0, L.stream, g, ph, cd); break;
    default: hipLaunchKernelGGL((k_sweep<ST, D, MODEL, 1, 0, 1>), grd, blk, 0, L.stream, g, ph, cd); break;
  }
  return hipGetLastError();
}

template <int ST>
hipError_t sweep_inj_t(const Launch& L, const Grid& g, const Phys& ph, const Codec& cd, int parity,
                       const float* dq, const int* flag) {
  const dim3 grd = cell_grid(g, L.block_x), blk(L.block_x);
  if (parity == 0)
    hipLaunchKernelGGL((k_sweep<ST, 2, 0, 0, 0, 0, true>), grd, blk, 0, L.stream, g, ph, cd, Body{}, dq, flag);
  else
    hipLaunchKernelGGL((k_sweep<ST, 2, 0, 1, 0, 0, true>), grd, blk, 0, L.stream, g, ph, cd, Body{}, dq, flag);
  return hipGetLastError();
}

template <int ST>
hipError_t boundary_t(const Launch& L, const Grid& g, const Phys& ph, const Codec& cd, int parity,
                      const Body* b, const Inflow* in, int what) {
  if (what == 0) {  // faces
    const long long area = std::max({(long long)g.ny * g.nz, (long long)g.nx * g.nz, (long long)g.nx * g.ny});
    hipLaunchKernelGGL((k_faces<ST>), dim3((unsigned)((area + 255) / 256), 1, 6), dim3(256), 0, L.stream, g, ph,
                       cd, parity, *in);
  } else if (what == 1) {  // sweep with the bounce-back body
    const dim3 grd = cell_grid(g, L.block_x), blk(L.block_x);
    switch ((ph.collision ? 2 : 0) + parity) {
      case 0: hipLaunchKernelGGL((k_sweep<ST, 3, 0, 0, 1, 0>), grd, blk, 0, L.stream, g, ph, cd, *b); break;
      case 1: hipLaunchKernelGGL((k_sweep<ST, 3, 0, 1, 1, 0>), grd, blk, 0, L.stream, g, ph, cd, *b); break;
      case 2: hipLaunchKernelGGL((k_sweep<ST, 3, 0, 0, 1, 1>), grd, blk, 0, L.stream, g, ph, cd, *b); break;
      default: hipLaunchKernelGGL((k_sweep<ST, 3, 0, 1, 1, 1>), grd, blk, 0, L.stream, g, ph, cd, *b); break;
    }
  } else if (what == 3) {
    // homogenized body: the plain sweep outside the body's box, then the homogenized
    // sweep of the box; the two update disjoint cells, each cell exactly once
    const dim3 grd = cell_grid(g, L.block_x), blk(L.block_x);
    const int bx = b->box[1] - b->box[0], by = b->box[3] - b->box[2], bz = b->box[5] - b->box[4];
    const bool box = bx > 0 && by > 0 && bz > 0;
    const dim3 bgrd((unsigned)((bx + L.block_x - 1) / L.block_x), (unsigned)by, (unsigned)bz);
    switch ((ph.collision ? 2 : 0) + parity) {
      case 0:
        hipLaunchKernelGGL((k_sweep<ST, 3, 0, 0, 3, 0>), grd, blk, 0, L.stream, g, ph, cd, *b);
        if (box) hipLaunchKernelGGL((k_sweep<ST, 3, 0, 0, 2, 0>), bgrd, blk, 0, L.stream, g, ph, cd, *b);
        break;
      case 1:
        hipLaunchKernelGGL((k_sweep<ST, 3, 0, 1, 3, 0>), grd, blk, 0, L.stream, g, ph, cd, *b);
        if (box) hipLaunchKernelGGL((k_sweep<ST, 3, 0, 1, 2, 0>), bgrd, blk, 0, L.stream, g, ph, cd, *b);
        break;
      case 2:
        hipLaunchKernelGGL((k_sweep<ST, 3, 0, 0, 3, 1>), grd, blk, 0, L.stream, g, ph, cd, *b);
        if (box) hipLaunchKernelGGL((k_sweep<ST, 3, 0, 0, 2, 1>), bgrd, blk, 0, L.stream, g, ph, cd, *b);
        break;
      default:
        hipLaunchKernelGGL((k_sweep<ST, 3, 0, 1, 3, 1>), grd, blk, 0, L.stream, g, ph, cd, *b);
        if (box) hipLaunchKernelGGL((k_sweep<ST, 3, 0, 1, 2, 1>), bgrd, blk, 0, L.stream, g, ph, cd, *b);
        break;
    }
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

// dispatch on (storage, dim, model) for functions templated <ST, D, MODEL>
template <template <int, int, int> class Fn, typename... A>
hipError_t dispatch(const Launch& L, A&&... args) {
  const int key = L.storage * 100 + L.dim * 10 + L.model;
  switch (key) {
#define VLBM_CASE(ST, D, M) \
  case ST * 100 + D * 10 + M: return Fn<ST, D, M>::run(L, args...);
    VLBM_CASE(0, 2, 0) VLBM_CASE(0, 3, 0) VLBM_CASE(0, 3, 1)
    VLBM_CASE(1, 2, 0) VLBM_CASE(1, 3, 0) VLBM_CASE(1, 3, 1)
    VLBM_CASE(2, 2, 0) VLBM_CASE(2, 3, 0) VLBM_CASE(2, 3, 1)
    VLBM_CASE(3, 2, 0) VLBM_CASE(3, 3, 0) VLBM_CASE(3, 3, 1)
#undef VLBM_CASE
    default: return hipErrorInvalidValue;
  }
}

template <int ST, int D, int M>
struct SweepFn {
  static hipError_t run(const Launch& L, const Grid& g, const Phys& ph, const Codec& cd, int par) {
    return sweep_t<ST, D, M>(L, g, ph, cd, par);
  }
};
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

hipError_t launch_sweep(const Launch& L, const Grid& g, const Phys& ph, const Codec& cd, int parity) {
  return dispatch<SweepFn>(L, g, ph, cd, parity);
}

hipError_t launch_init(const Launch& L, const Grid& g, const Phys& ph, const Codec& cd,
                       const void* Q, int q_is_f32) {
  return dispatch<InitFn>(L, g, ph, cd, Q, q_is_f32);
}

hipError_t launch_sweep_inj(const Launch& L, const Grid& g, const Phys& ph, const Codec& cd, int parity,
                            const float* dq, const int* flag) {
  if (L.dim != 2 || L.model != 0 || ph.collision != 0) return hipErrorInvalidValue;
  if (L.storage == ST_F32) return sweep_inj_t<ST_F32>(L, g, ph, cd, parity, dq, flag);
  if (L.storage == ST_F64) return sweep_inj_t<ST_F64>(L, g, ph, cd, parity, dq, flag);
  return hipErrorInvalidValue;
}

hipError_t launch_faces(const Launch& L, const Grid& g, const Phys& ph, const Codec& cd, int parity,
                        const Inflow& in) {
  return boundary(L, g, ph, cd, parity, nullptr, &in, 0);
}

hipError_t launch_sweep_body(const Launch& L, const Grid& g, const Phys& ph, const Codec& cd, int parity,
                             const Body& b, int mode) {
  if (mode == 2) return boundary(L, g, ph, cd, parity, &b, nullptr, 3);
  if (mode != 1 || !g.mask) return hipErrorInvalidValue;
  return boundary(L, g, ph, cd, parity, &b, nullptr, 1);
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
  if (L.dim == 2)
    hipLaunchKernelGGL((k_divc<2>), dim3(nblk), dim3(kReduceThreads), 0, L.stream, g, Qout, partial);
  else
    hipLaunchKernelGGL((k_divc<3>), dim3(nblk), dim3(kReduceThreads), 0, L.stream, g, Qout, partial);
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

// Internal: device helpers shared by the sweep (vlbm_sweep.hip) and the other
// kernels (vlbm_kernels.hip) -- storage codecs, periodic neighbours, scalar-base
// plane access, the body's geometry and field, and the (storage, dim, model)
// dispatch of the launchers.  Not installed.
#pragma once

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
// A scalar the compiler must treat as new at each use.  The FP64 decode converts the
// codec's FP32 constants to double; inside a grid-stride loop the compiler would
// otherwise hoist all 2 x K x Q converted constants out of the loop and keep them in
// VGPRs (over 300 for 26 variables: one wave per SIMD, and scratch spills).
__device__ __forceinline__ float opaque(float v) {
  asm volatile("" : "+v"(v));
  return v;
}

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
    return (double)opaque(cd.rest[j]) + (double)opaque(cd.sc[j]) * (double)h2f(v);
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
    return (double)opaque(cd.rest[j]) + (double)opaque(cd.sc[j]) * (double)b2f(v);
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
// A store one element off the wavefront's alignment (the +-x populations on parity 1)
// fills only part of its first and last cache lines; the neighbouring wavefront fills
// the rest.  With the ordinary cache policy L2 merges the two halves before writing the
// line back; the streaming policy sends the partial lines on (measured on the
// 26-variable sweep: parity 1 8.6 % faster with this store for those two planes).
template <typename T>
__device__ __forceinline__ void st_shifted(void* base, size_t plane_bytes, int plane, unsigned off, T v) {
  *(VLBM_GLOBAL T*)(plane_base(base, plane_bytes, plane) + off) = v;
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

dim3 cell_grid(const Grid& g, int bx) { return dim3((g.nx + bx - 1) / bx, g.ny, g.nz); }

// dispatch on (storage, dim, model) for functions templated <ST, D, MODEL>
template <template <int, int, int> class Fn, typename... A>
hipError_t dispatch(const Launch& L, A&&... args) {
  const int key = L.storage * 100 + L.dim * 10 + L.model;
  switch (key) {
#define VLBM_CASE(ST, D, M) \
  case ST * 100 + D * 10 + M: return Fn<ST, D, M>::run(L, args...);
    VLBM_CASE(0, 2, 0) VLBM_CASE(0, 3, 0) VLBM_CASE(0, 3, 1) VLBM_CASE(0, 2, 2) VLBM_CASE(0, 3, 2)
    VLBM_CASE(1, 2, 0) VLBM_CASE(1, 3, 0) VLBM_CASE(1, 3, 1) VLBM_CASE(1, 2, 2) VLBM_CASE(1, 3, 2)
    VLBM_CASE(2, 2, 0) VLBM_CASE(2, 3, 0) VLBM_CASE(2, 3, 1) VLBM_CASE(2, 2, 2) VLBM_CASE(2, 3, 2)
    VLBM_CASE(3, 2, 0) VLBM_CASE(3, 3, 0) VLBM_CASE(3, 3, 1) VLBM_CASE(3, 2, 2) VLBM_CASE(3, 3, 2)
    VLBM_CASE(0, 2, 3) VLBM_CASE(0, 3, 3) VLBM_CASE(1, 2, 3) VLBM_CASE(1, 3, 3)
    VLBM_CASE(2, 2, 3) VLBM_CASE(2, 3, 3) VLBM_CASE(3, 2, 3) VLBM_CASE(3, 3, 3)
    VLBM_CASE(0, 2, 4) VLBM_CASE(1, 2, 4) VLBM_CASE(2, 2, 4) VLBM_CASE(3, 2, 4)
#undef VLBM_CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace
}  // namespace vlbm

// The VLBM MHD sweep (gfx950): gather, decode, collide, encode, scatter, in place.
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
#include "vlbm_device.h"

namespace vlbm {
namespace {

// BODY (D3Q7 ideal): solid cells are skipped; a link i whose neighbour x + e_i is
// solid returns the post-collision population into direction opposite(i) of the
// same cell -- halfway bounce-back with the moving-wall flux correction for rho and
// E, anti-bounce-back to rho u_w and to the dipole field at the link midpoint for
// rho u and B.  In the AA layout that population belongs at slot i of cell x + e_i
// after a parity-0 step and at slot opposite(i) of x after a parity-1 step, places
// no other thread writes because the solid cell runs no update.
// INJ: before the collision add *dqflag * w_i dq[k][c] to f_{k,i} (the pending learned
// coarse correction, which shifts the zeroth moments by dq); dq is FP32 [K][N].
// Occupancy: the FP32 26-variable sweep needs 256 VGPRs + 26 AGPRs at parity 0,
// one wavefront per SIMD; bounding it to two per SIMD costs 48 B of scratch per lane
// and was measured 4-5 % faster (at parity 1 the bound spills more and is slower).
template <int ST, int D, int MODEL, int PAR, int BODY = 0, int COLL = 0, bool INJ = false>
__global__ __launch_bounds__(256, (MODEL == 1 && ST == ST_F32 && PAR == 0 && COLL == 0) ? 2 : 1) void k_sweep(const Grid g, const Phys ph, const Codec cd,
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

// what 1: the bounce-back body; 3: the homogenized body
template <int ST>
hipError_t sweep_body_t(const Launch& L, const Grid& g, const Phys& ph, const Codec& cd, int parity,
                        const Body* b, int what) {
  if (what == 1) {
    const dim3 grd = cell_grid(g, L.block_x), blk(L.block_x);
    switch ((ph.collision ? 2 : 0) + parity) {
      case 0: hipLaunchKernelGGL((k_sweep<ST, 3, 0, 0, 1, 0>), grd, blk, 0, L.stream, g, ph, cd, *b); break;
      case 1: hipLaunchKernelGGL((k_sweep<ST, 3, 0, 1, 1, 0>), grd, blk, 0, L.stream, g, ph, cd, *b); break;
      case 2: hipLaunchKernelGGL((k_sweep<ST, 3, 0, 0, 1, 1>), grd, blk, 0, L.stream, g, ph, cd, *b); break;
      default: hipLaunchKernelGGL((k_sweep<ST, 3, 0, 1, 1, 1>), grd, blk, 0, L.stream, g, ph, cd, *b); break;
    }
  } else {
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
  }
  return hipGetLastError();
}

template <int ST, int D, int M>
struct SweepFn {
  static hipError_t run(const Launch& L, const Grid& g, const Phys& ph, const Codec& cd, int par) {
    return sweep_t<ST, D, M>(L, g, ph, cd, par);
  }
};

}  // namespace

hipError_t launch_sweep(const Launch& L, const Grid& g, const Phys& ph, const Codec& cd, int parity) {
  return dispatch<SweepFn>(L, g, ph, cd, parity);
}

hipError_t launch_sweep_inj(const Launch& L, const Grid& g, const Phys& ph, const Codec& cd, int parity,
                            const float* dq, const int* flag) {
  if (L.dim != 2 || L.model != 0 || ph.collision != 0) return hipErrorInvalidValue;
  if (L.storage == ST_F32) return sweep_inj_t<ST_F32>(L, g, ph, cd, parity, dq, flag);
  if (L.storage == ST_F64) return sweep_inj_t<ST_F64>(L, g, ph, cd, parity, dq, flag);
  return hipErrorInvalidValue;
}

hipError_t launch_sweep_body(const Launch& L, const Grid& g, const Phys& ph, const Codec& cd, int parity,
                             const Body& b, int mode) {
  if (L.dim != 3 || L.model != 0) return hipErrorInvalidValue;
  if (mode != 2 && (mode != 1 || !g.mask)) return hipErrorInvalidValue;
  const int what = mode == 2 ? 3 : 1;
  switch (L.storage) {
    case ST_F64: return sweep_body_t<ST_F64>(L, g, ph, cd, parity, &b, what);
    case ST_F32: return sweep_body_t<ST_F32>(L, g, ph, cd, parity, &b, what);
    case ST_F16: return sweep_body_t<ST_F16>(L, g, ph, cd, parity, &b, what);
    case ST_BF16: return sweep_body_t<ST_BF16>(L, g, ph, cd, parity, &b, what);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace vlbm

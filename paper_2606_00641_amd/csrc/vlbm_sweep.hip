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

// Lane shifts across the 64-lane wavefront (DPP wave_shr:1 / wave_shl:1):
// lane_up(e, v) gives lane l the v of lane l - 1 and lane 0 its own e; lane_dn(e, v)
// gives lane l the v of lane l + 1 and lane 63 its own e.  A lane that is inactive
// at the shift is read as out of range (its neighbour gets e), so the shifts run with
// every lane of the wavefront active.
__device__ __forceinline__ unsigned up1(unsigned e, unsigned v) {
  return __builtin_amdgcn_update_dpp((int)e, (int)v, 0x138, 0xf, 0xf, false);
}
__device__ __forceinline__ unsigned dn1(unsigned e, unsigned v) {
  return __builtin_amdgcn_update_dpp((int)e, (int)v, 0x130, 0xf, 0xf, false);
}
template <bool UP, typename T>
__device__ __forceinline__ T lane_shift(T e, T v) {
  auto sh = [](unsigned ee, unsigned vv) { return UP ? up1(ee, vv) : dn1(ee, vv); };
  if constexpr (sizeof(T) == 8) {
    const unsigned long long ue = __builtin_bit_cast(unsigned long long, e);
    const unsigned long long uv = __builtin_bit_cast(unsigned long long, v);
    const unsigned long long r = (unsigned long long)sh((unsigned)ue, (unsigned)uv) |
                                 ((unsigned long long)sh((unsigned)(ue >> 32), (unsigned)(uv >> 32)) << 32);
    return __builtin_bit_cast(T, r);
  } else if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, sh(__builtin_bit_cast(unsigned, e), __builtin_bit_cast(unsigned, v)));
  } else {
    return (T)sh((unsigned)e, (unsigned)v);
  }
}

// Wavefront-edge values of the x planes, exchanged through LDS (a workgroup has at
// most 256 threads, four wavefronts); separate arrays for the pre- and post-collision
// exchange, so that a wavefront writing the second never overwrites a value another
// wavefront has yet to read from the first.
constexpr int kMaxWaves = 4;
template <typename T, int K, bool ON>
struct XchLds {
  T lo[2][kMaxWaves][K];  // lane 0's value of each wavefront
  T hi[2][kMaxWaves][K];  // lane 63's value
};
template <typename T, int K>
struct XchLds<T, K, false> {};

// Workgroups that share x rows (the lane exchanges of k_sweep and k_sweep2) are numbered
// along a 1-D grid, and the hardware deals them to the eight XCDs in turn by that
// number.  When several workgroups share a row (segments s = 0..S-1), the row's segments
// take numbers eight apart, 8 S q + 8 s + j for row 8 q + j, so they run on one XCD: the
// boundary elements two neighbouring segments both touch then meet in that XCD's L2
// instead of being fetched from HBM by two of them.
__device__ __forceinline__ void xcd_row_tile(int nseg, int nrows, int& seg, int& row) {
  const int L = (int)blockIdx.x;
  if (nseg == 1) {
    seg = 0;
    row = L;
    return;
  }
  const int q = L / (8 * nseg), rem = L - q * 8 * nseg;
  const int gsz = min(8, nrows - 8 * q);  // rows in this group (fewer in the last one)
  seg = rem / gsz;
  row = 8 * q + (rem - seg * gsz);
}


// XCH (parity 1, plain sweep, workgroups tiling every x row exactly): the +-x
// populations are read and written at the cell's own, aligned slots and passed
// between neighbouring lanes instead of being accessed one element off the
// wavefront's alignment.  Cell x needs f_{+x}(x) = slot(-x) of x - 1 and f_{-x}(x) =
// slot(+x) of x + 1: each lane loads its own slots(-x) and (+x) and takes the values
// of lanes l - 1 and l + 1; the post-collision f_{+x}(x) belongs to slot(+x) of
// x + 1 and f_{-x}(x) to slot(-x) of x - 1, so each lane stores the values of lanes
// l - 1 and l + 1 at its own slots.  Between wavefronts the edge values go through
// LDS; at the ends of a workgroup that spans a whole row they wrap around the row
// (periodic), else the end lanes read and write the neighbouring workgroup's cell
// directly, one element each.
// BODY 1 (D3Q7 ideal, every cell) and BODY 4 (the same over the body's box only, the
// grid offset by its corner as for BODY 2): solid cells are skipped; a link i whose
// neighbour x + e_i is solid returns the post-collision population into direction opposite(i) of the
// same cell -- halfway bounce-back with the moving-wall flux correction for rho and
// E, anti-bounce-back to rho u_w and to the dipole field at the link midpoint for
// rho u and B.  In the AA layout that population belongs at slot i of cell x + e_i
// after a parity-0 step and at slot opposite(i) of x after a parity-1 step, places
// no other thread writes because the solid cell runs no update.
// INJ: before the collision add w_i (dq[k][c] - mean[b][k]) to f_{k,i} when dqctl[0] is
// nonzero (the pending learned coarse correction, projected, which shifts the zeroth
// moments; dq FP32 [K][N], control block dqctl as launch_sweep_inj describes).
// Occupancy: the FP32 26-variable sweep needs 256 VGPRs + 26 AGPRs at parity 0,
// one wavefront per SIMD; bounding it to two per SIMD costs 48 B of scratch per lane
// and was measured 4-5 % faster (at parity 1 it spills 72 B per lane and, re-measured on
// the current kernel, changes nothing: 4.685-4.692 against 4.685-4.687 ms per step).  The
// FP16/BF16 13-component sweep at parity 1 is bounded to three wavefronts per SIMD (FP16
// 173 -> 151 VGPRs, no spill): with the XCD-grouped workgroup order of the lane exchange
// it then runs 12 % (FP16) and 14 % (BF16) faster on 4096^2 than with the row grid, where
// at two wavefronts per SIMD the same order had made FP16 19 % slower.
template <int ST, int D, int MODEL, int PAR, int BODY = 0, int COLL = 0, bool INJ = false, bool XCH = false,
          bool FX = false, int SRC = 0>
__global__ __launch_bounds__(256, (MODEL == 1 && ST == ST_F32 && PAR == 0 && COLL == 0)
                                      ? 2
                                      : ((MODEL == 4 && (ST == ST_F16 || ST == ST_BF16) && PAR == 1 && COLL == 0) ? 3 : 1))
    void k_sweep(
    const Grid g, const Phys ph, const Codec cd, const Body bd, const float* __restrict__ dq,
    const int* __restrict__ dqctl, const Inflow in, const MomentsOut mo) {
  using S = Store<ST>;
  using T = typename S::T;
  using R = typename S::R;
  constexpr int NQ = 2 * D + 1;
  constexpr int K = kNVars<MODEL>;
  constexpr unsigned ES = sizeof(T);
  static_assert(!XCH || (PAR == 1 && (BODY == 0 || BODY == 3)), "lane exchange: plain sweep at parity 1");
  static_assert(!FX || (D == 3 && MODEL == 0 && BODY != 2 && BODY != 4 && !INJ), "x faces: D3Q7 ideal MHD");
  constexpr bool kBB = BODY == 1 || BODY == 4;     // link-wise bounce-back (mask)
  constexpr bool kInBox = BODY == 2 || BODY == 4;  // grid over the body's box
  __shared__ XchLds<T, K, XCH> xl;
  // BODY 2 runs over the body's box only (grid = box extent, offset by its corner);
  // BODY 3 is the plain sweep of every other cell.
  int x, y, z;
  if constexpr (XCH) {
    int seg, rw;
    xcd_row_tile(g.nx / (int)blockDim.x, g.ny * g.nz, seg, rw);
    x = seg * (int)blockDim.x + (int)threadIdx.x;
    y = rw % g.ny;
    z = rw / g.ny;
  } else {
    x = blockIdx.x * blockDim.x + threadIdx.x;
    y = blockIdx.y;
    z = blockIdx.z;
  }
  if constexpr (kInBox) {
    x += bd.box[0];
    y += bd.box[2];
    z += bd.box[4];
    if (x >= bd.box[1]) return;
  } else {
    if (x >= g.nx) return;
  }
  // with the lane exchange, a cell of the body's box still takes part (its lane
  // relays its own x slots to the neighbour lanes) but updates nothing
  bool own = true, own_l = true, own_r = true;
  if constexpr (BODY == 3) {
    auto in_box = [&](int xx) {
      return xx >= bd.box[0] && xx < bd.box[1] && y >= bd.box[2] && y < bd.box[3] && z >= bd.box[4] && z < bd.box[5];
    };
    if constexpr (XCH) {
      own = !in_box(x);
      own_l = !in_box(x == 0 ? g.nx - 1 : x - 1);
      own_r = !in_box(x + 1 == g.nx ? 0 : x + 1);
    } else {
      if (in_box(x)) return;
    }
  }
  (void)own;
  (void)own_l;
  (void)own_r;
  const unsigned c = (unsigned)x + (unsigned)g.nx * ((unsigned)y + (unsigned)g.ny * (unsigned)z);
  void* const F = g.f;
  // PK: 16-bit storage of the 26-variable model keeps variables 2p and 2p + 1 of a slot in
  // one 32-bit element (Grid::pk), so every access moves 4 bytes per lane; both halves
  // stream in the same direction, so the in-place pattern is unchanged
  constexpr bool PK = MODEL == 1 && (ST == ST_F16 || ST == ST_BF16) && !XCH;
  constexpr unsigned EA = PK ? 4u : ES;  // bytes per addressed element
  const size_t pb = (size_t)g.stride * EA;
  unsigned mk = 0;
  if constexpr (kBB) {
    mk = g.mask[c];
    if (mk & kSolid) return;
  }

  // byte offsets of this cell and of its neighbours x + e_a (np), x - e_a (nm)
  unsigned np[3], nm[3];
  if constexpr (PAR == 1 || kBB) {
    neighbours<D>(g, x, y, z, c, np, nm);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      np[a] *= EA;
      nm[a] *= EA;
    }
  }
  const unsigned co = c * EA;

  R f[K][NQ];
  T raw[XCH ? K : 1][2];
  (void)raw;
  if constexpr (PK) {
#pragma unroll
    for (int p = 0; p < K / 2; ++p)
#pragma unroll
      for (int i = 0; i < NQ; ++i) {
        unsigned w;
        if constexpr (PAR == 0) {
          w = ld<unsigned>(F, pb, p * NQ + i, co);
        } else {
          const unsigned src = (i == 0) ? co : ((i & 1) ? nm[(i - 1) >> 1] : np[(i - 1) >> 1]);
          w = ld<unsigned>(F, pb, p * NQ + opposite(i), src);
        }
        f[2 * p][i] = S::dec((T)(w & 0xffffu), cd, 2 * p * NQ + i);
        f[2 * p + 1][i] = S::dec((T)(w >> 16), cd, (2 * p + 1) * NQ + i);
      }
  }
#pragma unroll
  for (int k = 0; k < (PK ? 0 : K); ++k) {
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      T v;
      if constexpr (PAR == 0) {
        v = ld<T>(F, pb, k * NQ + i, co);
      } else if constexpr (XCH) {
        // i = 1, 2: this cell's own slot opposite(i), handed to the neighbour lane below
        const unsigned src = (i <= 2) ? co : ((i & 1) ? nm[(i - 1) >> 1] : np[(i - 1) >> 1]);
        v = ld<T>(F, pb, k * NQ + opposite(i), src);
      } else {
        // f_i(x) was written by cell x - e_i into its slot opposite(i)
        const unsigned src = (i == 0) ? co : ((i & 1) ? nm[(i - 1) >> 1] : np[(i - 1) >> 1]);
        v = ld<T>(F, pb, k * NQ + opposite(i), src);
      }
      if constexpr (XCH) {
        if (i == 1 || i == 2) {
          raw[k][i - 1] = v;
          continue;
        }
      }
      f[k][i] = S::dec(v, cd, k * NQ + i);
    }
  }
  if constexpr (XCH) {
    // raw[k][0] = slot(-x) of x (f_{+x} of x + 1), raw[k][1] = slot(+x) of x (f_{-x} of x - 1)
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, nw = (int)(blockDim.x >> 6);
    const bool row = (int)blockDim.x == g.nx;
    if (lane == 63) {
#pragma unroll
      for (int k = 0; k < K; ++k) xl.hi[0][w][k] = raw[k][0];
    }
    if (lane == 0) {
#pragma unroll
      for (int k = 0; k < K; ++k) xl.lo[0][w][k] = raw[k][1];
    }
    __syncthreads();
    // what lane 0 needs from the left and lane 63 from the right: another wavefront's
    // edge value, or (ends of a workgroup that does not span the row) the
    // neighbouring workgroup's cell, at a wavefront-uniform address
    const unsigned rowc = (unsigned)g.nx * ((unsigned)y + (unsigned)g.ny * (unsigned)z);
    const unsigned x0 = (unsigned)(x - t), x1 = x0 + blockDim.x;
    const unsigned cl = (rowc + (x0 == 0 ? (unsigned)g.nx - 1u : x0 - 1u)) * ES;
    const unsigned cr = (rowc + (x1 == (unsigned)g.nx ? 0u : x1)) * ES;
    T el[K], er[K];
    if (w > 0 || row) {
#pragma unroll
      for (int k = 0; k < K; ++k) el[k] = xl.hi[0][w > 0 ? w - 1 : nw - 1][k];
    } else {
#pragma unroll
      for (int k = 0; k < K; ++k) el[k] = ld<T>(F, pb, k * NQ + 2, cl);
    }
    if (w < nw - 1 || row) {
#pragma unroll
      for (int k = 0; k < K; ++k) er[k] = xl.lo[0][w < nw - 1 ? w + 1 : 0][k];
    } else {
#pragma unroll
      for (int k = 0; k < K; ++k) er[k] = ld<T>(F, pb, k * NQ + 1, cr);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      f[k][1] = S::dec(lane_shift<true>(el[k], raw[k][0]), cd, k * NQ + 1);
      f[k][2] = S::dec(lane_shift<false>(er[k], raw[k][1]), cd, k * NQ + 2);
    }
  }

  if constexpr (FX) {
    // Static x faces (Sec. 2.4) inside the sweep: a node of a non-periodic x face
    // that lies on no other non-periodic face takes f := f^eq(Q_bc) before it
    // collides -- Q_bc the inflow state, or (zero gradient) the moments of its
    // neighbour x +- 1 in the same row, which the neighbour lane holds.  This is what
    // the separate face pass computes (same moment order, same storage rounding of
    // f^eq) without its one-element-per-row accesses; the y and z faces, edges
    // included, stay with that pass.
    R q[8], ql[8], qr[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      R a = R(0);
#pragma unroll
      for (int i = 0; i < NQ; ++i) a += f[k][i];
      q[k] = a;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      ql[k] = lane_shift<true>(q[k], q[k]);   // moments of x - 1
      qr[k] = lane_shift<false>(q[k], q[k]);  // moments of x + 1
    }
    const bool yin = g.bc[2] == 0 || (y > 0 && y < g.ny - 1);
    const bool zin = g.bc[4] == 0 || (z > 0 && z < g.nz - 1);
    const int side = x == 0 ? 0 : (x == g.nx - 1 ? 1 : -1);
    if (side >= 0 && g.bc[side] != 0 && yin && zin) {
      R Qb[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) Qb[k] = g.bc[side] == 1 ? R(in.q[k]) : (side == 0 ? qr[k] : ql[k]);
      R Jb[3] = {R(0), R(0), R(0)};
      R P[8][3], Sv[8], dlb;
      flux_source<R, 3, 0>(Qb, Jb, ph, P, Sv, dlb);
      const R wi = R(ph.wi);
      const R w0 = rest_weight<R, 3>(wi);
#pragma unroll
      for (int k = 0; k < 8; ++k)
#pragma unroll
        for (int i = 0; i < NQ; ++i)
          f[k][i] = S::dec(S::enc(feq_dir<R, 3>(Qb[k], P[k], i, w0, wi), cd, k * NQ + i), cd, k * NQ + i);
    }
  }

  if constexpr (INJ) {
    if (dqctl[0]) {
      const size_t N = (size_t)g.nx * g.ny * g.nz;
      const R wi = R(ph.wi);
      const R w0 = rest_weight<R, D>(wi);
      const int* __restrict__ mean = dqctl + 1 + 8 * inj_lattice(D, z);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const R d = (R)(dq[(size_t)k * N + c] - __int_as_float(mean[k]));
#pragma unroll
        for (int i = 0; i < NQ; ++i) f[k][i] += (i == 0 ? w0 : wi) * d;
      }
    }
  }

  R dl;
  if constexpr (!kBB) {
    if constexpr (BODY == 2) {
      static_assert(D == 3 && MODEL == 0, "homogenized body: D3Q7 ideal MHD");
      R Q[K], pt;
      const bool near = HlbmTarget::near_body(bd, x, y, z);
      collide<R, D, MODEL, COLL>(f, ph, dl, Q, pt, HlbmTarget{&bd, x, y, z, near, ph.s, ph.gm1});
    } else if constexpr (INJ && MODEL == 0) {
      R Q[K], pt;
      collide<R, D, MODEL, COLL>(f, ph, dl, Q, pt);
      if (mo.x) {  // the moments the next network evaluation takes
        const size_t N = (size_t)g.nx * g.ny * g.nz;
        unsigned h[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const float xq = (float)Q[k];
          mo.x[(size_t)k * N + c] = xq;
          const unsigned u = __float_as_uint((xq - mo.mean[k]) * mo.istd[k]);
          h[k] = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;  // BF16, nearest even
        }
        *reinterpret_cast<uint4*>(mo.act + (size_t)c * K) =
            make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16));
      }
    } else if constexpr (SRC == 2) {
      // Chai's source: the cell's previous source in, this step's out (own cell, any parity)
      const size_t N = (size_t)g.nx * g.ny * g.nz;
      R* __restrict__ sprev = static_cast<R*>(g.sprev);
      R sp[K], Q[K], pt;
#pragma unroll
      for (int k = 0; k < K; ++k) sp[k] = sprev[(size_t)k * N + c];
      collide<R, D, MODEL, COLL, NoTarget, SRC>(f, ph, dl, Q, pt, NoTarget{}, sp);
#pragma unroll
      for (int k = 0; k < K; ++k) sprev[(size_t)k * N + c] = sp[k];
    } else if constexpr (SRC == 1) {
      R Q[K], pt;
      collide<R, D, MODEL, COLL, NoTarget, SRC>(f, ph, dl, Q, pt);
    } else {
      collide<R, D, MODEL, COLL>(f, ph, dl);
    }
    if constexpr (PK) {
#pragma unroll
      for (int p = 0; p < K / 2; ++p)
#pragma unroll
        for (int i = 0; i < NQ; ++i) {
          const unsigned w = (unsigned)S::enc(f[2 * p][i], cd, 2 * p * NQ + i) |
                             ((unsigned)S::enc(f[2 * p + 1][i], cd, (2 * p + 1) * NQ + i) << 16);
          if constexpr (PAR == 0) {
            st<unsigned>(F, pb, p * NQ + opposite(i), co, w);
          } else {
            const unsigned dst = (i == 0) ? co : ((i & 1) ? np[(i - 1) >> 1] : nm[(i - 1) >> 1]);
            if (i == 1 || i == 2)
              st_shifted<unsigned>(F, pb, p * NQ + i, dst, w);
            else
              st<unsigned>(F, pb, p * NQ + i, dst, w);
          }
        }
    }
#pragma unroll
    for (int k = 0; k < (PK ? 0 : K); ++k) {
#pragma unroll
      for (int i = 0; i < NQ; ++i) {
        if constexpr (XCH) {
          if (i == 1 || i == 2 || !own) continue;
        }
        const T v = S::enc(f[k][i], cd, k * NQ + i);
        if constexpr (PAR == 0) {
          st<T>(F, pb, k * NQ + opposite(i), co, v);
        } else {
          const unsigned dst = (i == 0) ? co : ((i & 1) ? np[(i - 1) >> 1] : nm[(i - 1) >> 1]);
          if (i == 1 || i == 2)
            st_shifted<T>(F, pb, k * NQ + i, dst, v);
          else
            st<T>(F, pb, k * NQ + i, dst, v);
        }
      }
    }
    if constexpr (XCH) {
      // post-collision f_{+x}(x) -> slot(+x) of x + 1, f_{-x}(x) -> slot(-x) of x - 1,
      // each stored by the lane of that cell
      const int t = threadIdx.x, lane = t & 63, w = t >> 6, nw = (int)(blockDim.x >> 6);
      const bool row = (int)blockDim.x == g.nx;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        raw[k][0] = S::enc(f[k][1], cd, k * NQ + 1);
        raw[k][1] = S::enc(f[k][2], cd, k * NQ + 2);
      }
      if (lane == 63) {
#pragma unroll
        for (int k = 0; k < K; ++k) xl.hi[1][w][k] = raw[k][0];
      }
      if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) xl.lo[1][w][k] = raw[k][1];
      }
      __syncthreads();
      const int wl = w > 0 ? w - 1 : nw - 1, wr = w < nw - 1 ? w + 1 : 0;
      // ends of a workgroup that does not span the row: its last lane writes slot(+x)
      // of the next workgroup's first cell and its first lane slot(-x) of the previous
      // workgroup's last cell, whose own lanes skip those slots
      if (!row && own && t == (int)blockDim.x - 1) {
#pragma unroll
        for (int k = 0; k < K; ++k) st_shifted<T>(F, pb, k * NQ + 1, np[0], raw[k][0]);
      }
      if (!row && own && t == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) st_shifted<T>(F, pb, k * NQ + 2, nm[0], raw[k][1]);
      }
      // the lane shifts read every lane, so they run with all lanes active
#pragma unroll
      for (int k = 0; k < K; ++k) {
        raw[k][0] = lane_shift<true>(xl.hi[1][wl][k], raw[k][0]);
        raw[k][1] = lane_shift<false>(xl.lo[1][wr][k], raw[k][1]);
      }
      // slot(+x) takes the left neighbour's value, slot(-x) the right one's: stored
      // only where that neighbour was updated here
      if ((row || t != 0) && own_l) {
#pragma unroll
        for (int k = 0; k < K; ++k) st<T>(F, pb, k * NQ + 1, co, raw[k][0]);
      }
      if ((row || t != (int)blockDim.x - 1) && own_r) {
#pragma unroll
        for (int k = 0; k < K; ++k) st<T>(F, pb, k * NQ + 2, co, raw[k][1]);
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
          else if (i == 1 || i == 2)
            st_shifted<T>(F, pb, k * NQ + i, dst, v);
          else
            st<T>(F, pb, k * NQ + i, dst, v);
        }
      }
    }
  }
}

// Two cells per lane (FP16/BF16 storage; the plain sweep, or with the BOX and FX forms
// below the open D3Q7 lattice of the homogenized body): lane l of the workgroup that takes
// segment b of a row takes cells x0 = 2 (b B + l) and x0 + 1 (B threads per workgroup,
// 2 B cells per segment), so every plane access moves the 32-bit word of the
// pair -- the low half is cell x0.  A wavefront instruction that moves 2 bytes per lane
// runs far below HBM bandwidth on gfx950 (a streaming copy measured about 3 TB/s at 16
// bits per lane against 5 TB/s at 32).  Each cell is decoded, collided and encoded as
// in k_sweep: the same arithmetic, which the compiler may contract into fused
// multiply-adds differently in the two kernels, so they agree to one rounding of the
// stored value; the tilings of k_sweep2 agree bitwise.
// Parity 1 reads f_{+x}(x) from slot(-x) of x - 1 and f_{-x}(x) from slot(+x) of x + 1:
// a lane loads its own words of those slots, A = slot(-x)[x0, x0 + 1] and
// W = slot(+x)[x0, x0 + 1], and forms its pairs from the neighbour lanes' words,
// f_{+x} = (A of lane l - 1).hi : A.lo and f_{-x} = W.hi : (W of lane l + 1).lo; the
// post-collision f_{+x} pair goes to slot(+x) of x0 + 1, x0 + 2 and the f_{-x} pair to
// slot(-x) of x0 - 1, x0, so a lane stores at its own word (left lane's f_{+x}).hi :
// f_{+x}.lo and f_{-x}.hi : (right lane's f_{-x}).lo.  Between wavefronts the edge words
// go through LDS; at the ends of a workgroup that spans its row they wrap around the
// row, else the end lanes read the neighbouring workgroup's boundary element, and
// write the half that belongs to it, with 16-bit accesses (as k_sweep's lane exchange).
// BOX: the sweep of every cell outside the body's box (k_sweep's BODY 3); a cell of the
// box still loads and relays its words but stores nothing of its own.
// FX: the non-periodic x faces re-set inside the sweep as in k_sweep; x = 0 is the low
// cell of its lane and x = nx - 1 the high one, so the zero-gradient neighbour is the
// lane's other cell.  The workgroups are numbered by xcd_row_tile.
template <int ST, int D, int MODEL, int PAR, int COLL, bool BOX = false, bool FX = false>
__global__ __launch_bounds__(256) void k_sweep2(const Grid g, const Phys ph, const Codec cd, const Body bd,
                                                const Inflow in) {
  static_assert(ST == ST_F16 || ST == ST_BF16, "two cells per lane: 16-bit storage");
  static_assert(!(BOX || FX) || (D == 3 && MODEL == 0), "body box, x faces: D3Q7 ideal MHD");
  using S = Store<ST>;
  using R = typename S::R;
  using H = typename S::T;
  constexpr int NQ = 2 * D + 1;
  constexpr int K = kNVars<MODEL>;
  __shared__ XchLds<unsigned, K, true> xl;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, nw = (int)(blockDim.x >> 6);
  int seg, rw;
  xcd_row_tile(g.nx / (2 * (int)blockDim.x), g.ny * g.nz, seg, rw);
  const int y = rw % g.ny, z = rw / g.ny;
  const int x0 = 2 * (seg * (int)blockDim.x + t);
  const bool row = 2 * (int)blockDim.x == g.nx;
  const unsigned rowc = (unsigned)g.nx * ((unsigned)y + (unsigned)g.ny * (unsigned)z);
  const unsigned c = rowc + (unsigned)x0;
  void* const F = g.f;
  const size_t pb = (size_t)g.stride * sizeof(H);
  const unsigned co = c * (unsigned)sizeof(H);
  unsigned np[3], nm[3];
  if constexpr (PAR == 1) {
    neighbours<D>(g, x0, y, z, c, np, nm);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      np[a] *= (unsigned)sizeof(H);
      nm[a] *= (unsigned)sizeof(H);
    }
  }
  // byte offsets of the elements just outside this workgroup's stretch of the row
  const unsigned xa = (unsigned)(2 * seg * (int)blockDim.x), xb = xa + 2 * blockDim.x;
  const unsigned cl = (rowc + (xa == 0 ? (unsigned)g.nx - 1u : xa - 1u)) * (unsigned)sizeof(H);
  const unsigned cr = (rowc + (xb == (unsigned)g.nx ? 0u : xb)) * (unsigned)sizeof(H);

  unsigned P[K][NQ];  // the pair's words: low half cell x0, high half x0 + 1
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      if constexpr (PAR == 0) {
        P[k][i] = ld<unsigned>(F, pb, k * NQ + i, co);
      } else {
        // i = 1, 2: this pair's own slot opposite(i), combined with a neighbour lane's below
        const unsigned src = (i <= 2) ? co : ((i & 1) ? nm[(i - 1) >> 1] : np[(i - 1) >> 1]);
        P[k][i] = ld<unsigned>(F, pb, k * NQ + opposite(i), src);
      }
    }
  if constexpr (PAR == 1) {
    if (lane == 63) {
#pragma unroll
      for (int k = 0; k < K; ++k) xl.hi[0][w][k] = P[k][1];
    }
    if (lane == 0) {
#pragma unroll
      for (int k = 0; k < K; ++k) xl.lo[0][w][k] = P[k][2];
    }
    __syncthreads();
    unsigned el[K], er[K];  // lane 0's left word (its high half used), lane 63's right word (low half)
    if (w > 0 || row) {
#pragma unroll
      for (int k = 0; k < K; ++k) el[k] = xl.hi[0][w > 0 ? w - 1 : nw - 1][k];
    } else {
#pragma unroll
      for (int k = 0; k < K; ++k) el[k] = (unsigned)ld<H>(F, pb, k * NQ + 2, cl) << 16;
    }
    if (w < nw - 1 || row) {
#pragma unroll
      for (int k = 0; k < K; ++k) er[k] = xl.lo[0][w < nw - 1 ? w + 1 : 0][k];
    } else {
#pragma unroll
      for (int k = 0; k < K; ++k) er[k] = (unsigned)ld<H>(F, pb, k * NQ + 1, cr);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const unsigned left = lane_shift<true>(el[k], P[k][1]), right = lane_shift<false>(er[k], P[k][2]);
      P[k][1] = __builtin_amdgcn_alignbyte(P[k][1], left, 2);   // left.hi : A.lo
      P[k][2] = __builtin_amdgcn_alignbyte(right, P[k][2], 2);  // W.hi : right.lo
    }
  }

  bool inb[2] = {false, false};  // the cell lies in the body's box
  if constexpr (BOX) {
    const bool yz = y >= bd.box[2] && y < bd.box[3] && z >= bd.box[4] && z < bd.box[5];
    inb[0] = yz && x0 >= bd.box[0] && x0 < bd.box[1];
    inb[1] = yz && x0 + 1 >= bd.box[0] && x0 + 1 < bd.box[1];
  }
  bool face[2] = {false, false};  // x-face node on no other non-periodic face
  R qn[FX ? 8 : 1];               // zero gradient: the moments of the lane's other cell
  (void)qn;
  if constexpr (FX) {
    const bool yin = g.bc[2] == 0 || (y > 0 && y < g.ny - 1);
    const bool zin = g.bc[4] == 0 || (z > 0 && z < g.nz - 1);
    face[0] = x0 == 0 && g.bc[0] != 0 && yin && zin;
    face[1] = x0 + 1 == g.nx - 1 && g.bc[1] != 0 && yin && zin;
    if (face[0] || face[1]) {
      const int sh = face[0] ? 16 : 0;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        R a = R(0);
#pragma unroll
        for (int i = 0; i < NQ; ++i) a += S::dec((H)(P[k][i] >> sh), cd, k * NQ + i);
        qn[k] = a;
      }
    }
  }

  // the two cells, one after the other; each result replaces the half it came from
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    R f[K][NQ];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int i = 0; i < NQ; ++i) f[k][i] = S::dec((H)(P[k][i] >> (16 * j)), cd, k * NQ + i);
    if constexpr (FX) {
      if (face[j]) {
        const int side = j;  // x = 0 is always a low cell, x = nx - 1 a high one
        R Qb[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) Qb[k] = g.bc[side] == 1 ? R(in.q[k]) : qn[k];
        R Jb[3] = {R(0), R(0), R(0)};
        R Pf[8][3], Sv[8], dlb;
        flux_source<R, 3, 0>(Qb, Jb, ph, Pf, Sv, dlb);
        const R wi = R(ph.wi);
        const R w0 = rest_weight<R, 3>(wi);
#pragma unroll
        for (int k = 0; k < 8; ++k)
#pragma unroll
          for (int i = 0; i < NQ; ++i)
            f[k][i] = S::dec(S::enc(feq_dir<R, 3>(Qb[k], Pf[k], i, w0, wi), cd, k * NQ + i), cd, k * NQ + i);
      }
    }
    R dl;
    collide<R, D, MODEL, COLL>(f, ph, dl);
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int i = 0; i < NQ; ++i) {
        const unsigned h = (unsigned)S::enc(f[k][i], cd, k * NQ + i);
        P[k][i] = j == 0 ? (P[k][i] & 0xffff0000u) | h : (P[k][i] & 0xffffu) | (h << 16);
      }
  }

  // BOX: a slot whose owner -- the cell whose outgoing population it receives -- lies in
  // the box is not written (the box sweep that follows reads and writes it), so a word
  // with one such half is stored as its other half.  own0/own1: cells x0, x0 + 1;
  // ownl/ownr: the cells x0 - 1 and x0 + 2 whose populations the x-exchange words also
  // carry.  The choice between the two store sequences is made once per wavefront:
  // wavefronts that touch no box cell run the plain word stores as one straight block
  // (a test per store split them into blocks of their own and made the sweep 30-50 % slower).
  bool own0 = true, own1 = true, ownl = true, ownr = true, careful = false;
  if constexpr (BOX) {
    const bool yz = y >= bd.box[2] && y < bd.box[3] && z >= bd.box[4] && z < bd.box[5];
    const int xl = x0 == 0 ? g.nx - 1 : x0 - 1, xr = x0 + 2 == g.nx ? 0 : x0 + 2;
    own0 = !inb[0];
    own1 = !inb[1];
    ownl = !(yz && xl >= bd.box[0] && xl < bd.box[1]);
    ownr = !(yz && xr >= bd.box[0] && xr < bd.box[1]);
    careful = __builtin_amdgcn_ballot_w64(!(own0 && own1 && ownl && ownr)) != 0;
  }
  (void)ownl;
  (void)ownr;
  (void)careful;
  auto put = [&](auto cf, int plane, unsigned off, unsigned v, bool lo, bool hi) {
    if constexpr (decltype(cf)::value) {
      if (lo && hi)
        st<unsigned>(F, pb, plane, off, v);
      else if (lo)
        st_shifted<H>(F, pb, plane, off, (H)v);
      else if (hi)
        st_shifted<H>(F, pb, plane, off + (unsigned)sizeof(H), (H)(v >> 16));
    } else {
      st<unsigned>(F, pb, plane, off, v);
    }
  };
  // every store but the parity-1 x slots
  auto own_stores = [&](auto cf) {
    if constexpr (PAR == 0) {
#pragma unroll
      for (int k = 0; k < K; ++k)
#pragma unroll
        for (int i = 0; i < NQ; ++i) put(cf, k * NQ + opposite(i), co, P[k][i], own0, own1);
    } else {
#pragma unroll
      for (int k = 0; k < K; ++k)
#pragma unroll
        for (int i = 0; i < NQ; ++i) {
          if (i == 1 || i == 2) continue;
          const unsigned dst = (i == 0) ? co : ((i & 1) ? np[(i - 1) >> 1] : nm[(i - 1) >> 1]);
          put(cf, k * NQ + i, dst, P[k][i], own0, own1);
        }
    }
  };
  if constexpr (BOX) {
    if (careful)
      own_stores(std::true_type{});
    else
      own_stores(std::false_type{});
  } else {
    own_stores(std::false_type{});
  }

  if constexpr (PAR == 1) {
    if (lane == 63) {
#pragma unroll
      for (int k = 0; k < K; ++k) xl.hi[1][w][k] = P[k][1];
    }
    if (lane == 0) {
#pragma unroll
      for (int k = 0; k < K; ++k) xl.lo[1][w][k] = P[k][2];
    }
    __syncthreads();
    const int wl = w > 0 ? w - 1 : nw - 1, wr = w < nw - 1 ? w + 1 : 0;
    // the lane shifts read every lane, so they run with all lanes active
    unsigned left[K], right[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      left[k] = lane_shift<true>(xl.hi[1][wl][k], P[k][1]);
      right[k] = lane_shift<false>(xl.lo[1][wr][k], P[k][2]);
    }
    const bool first = !row && t == 0, last = !row && t == (int)blockDim.x - 1;
    auto x_stores = [&](auto cf) {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const unsigned vp = __builtin_amdgcn_alignbyte(P[k][1], left[k], 2);   // slot(+x) of x0, x0 + 1
        const unsigned vm = __builtin_amdgcn_alignbyte(right[k], P[k][2], 2);  // slot(-x) of x0, x0 + 1
        if (first) {
          // x0 - 1 is the previous workgroup's: it writes slot(+x) of x0; this lane writes
          // x0 + 1's, and slot(-x) of x0 - 1 (its own f_{-x}(x0))
          if (own0) {
            st_shifted<H>(F, pb, k * NQ + 1, co + (unsigned)sizeof(H), (H)(vp >> 16));
            st_shifted<H>(F, pb, k * NQ + 2, cl, (H)P[k][2]);
          }
        } else {
          put(cf, k * NQ + 1, co, vp, ownl, own0);
        }
        if (last) {
          // x0 + 2 is the next workgroup's: this lane writes slot(-x) of x0 only, and
          // slot(+x) of x0 + 2 (its own f_{+x}(x0 + 1))
          if (own1) {
            st_shifted<H>(F, pb, k * NQ + 2, co, (H)vm);
            st_shifted<H>(F, pb, k * NQ + 1, cr, (H)(P[k][1] >> 16));
          }
        } else {
          put(cf, k * NQ + 2, co, vm, own1, ownr);
        }
      }
    };
    if constexpr (BOX) {
      if (careful)
        x_stores(std::true_type{});
      else
        x_stores(std::false_type{});
    } else {
      x_stores(std::false_type{});
    }
  }
}

// The parity-1 lane exchange needs every workgroup to cover whole wavefronts of one
// x row (no partial workgroup, so that every lane reaches the barriers).  It is used
// for the 8-variable (and 5-variable) sweeps (measured on 512^3: parity 1 11-20 % faster in FP32,
// 12 % FP16, 10 % BF16); the 26-variable sweep runs one wavefront per SIMD, where the
// workgroup barrier leaves the CU idle, and was 16 % slower with it.
inline bool lane_exchange(const Grid& g, int block_x, int model) {
  return model != 1 && block_x % 64 == 0 && g.nx % block_x == 0;
}

// One k_sweep launch with the template flags chosen at run time: parity, collision
// (BGK or two-rate), lane exchange, x faces.  Only the combinations a caller can ask
// for are instantiated.
template <int ST, int D, int MODEL, int BODY, bool INJ>
void launch_k(const Launch& L, dim3 grd, int parity, int coll, bool xch, bool fx, const Grid& g, const Phys& ph,
              const Codec& cd, const Body& b, const float* dq, const int* flag, const Inflow& in,
              const MomentsOut& mo = MomentsOut{}) {
  constexpr bool kX = MODEL != 1 && (BODY == 0 || BODY == 3);  // exchange possible
  constexpr bool kF = D == 3 && MODEL == 0 && BODY != 2 && BODY != 4 && !INJ;  // x faces possible
  constexpr bool kC = !INJ;                                      // two-rate collisions possible
  auto go = [&](auto par_c, auto coll_c, auto xch_c, auto fx_c) {
    constexpr int P = decltype(par_c)::value, C = decltype(coll_c)::value;
    constexpr bool X = decltype(xch_c)::value, FXv = decltype(fx_c)::value;
    // the lane exchange numbers its workgroups along a 1-D grid (xcd_row_tile)
    const dim3 grid = X ? dim3((unsigned)((long long)(g.nx / L.block_x) * g.ny * g.nz)) : grd;
    hipLaunchKernelGGL((k_sweep<ST, D, MODEL, P, BODY, C, INJ, X, FXv>), grid, dim3(L.block_x), 0, L.stream, g, ph,
                       cd, b, dq, flag, in, mo);
  };
  using I0 = std::integral_constant<int, 0>;
  using I1 = std::integral_constant<int, 1>;
  using BF = std::false_type;
  using BT = std::true_type;
  auto with_fx = [&](auto par_c, auto coll_c, auto xch_c) {
    if constexpr (kF) {
      if (fx) return go(par_c, coll_c, xch_c, BT{});
    }
    go(par_c, coll_c, xch_c, BF{});
  };
  auto with_coll = [&](auto par_c, auto xch_c) {
    if constexpr (kC) {
      if (coll) return with_fx(par_c, I1{}, xch_c);
    }
    with_fx(par_c, I0{}, xch_c);
  };
  if (parity == 0) return with_coll(I0{}, BF{});
  if constexpr (kX) {
    if (xch) return with_coll(I1{}, BT{});
  }
  with_coll(I1{}, BF{});
}

// Sweeps with the Guo or Chai source operator: the plain periodic sweep (direct +-x
// accesses at parity 1), BGK or the moment-rate collisions, FP64/FP32 storage and the
// models with sources (ideal, resistive, 13-component); the library refuses the rest.
template <int ST, int D, int MODEL>
hipError_t sweep_src_t(const Launch& L, const Grid& g, const Phys& ph, const Codec& cd, int parity) {
  if constexpr ((ST == ST_F64 || ST == ST_F32) && (MODEL == 0 || MODEL == 1 || MODEL == 4)) {
    const dim3 grd = cell_grid(g, L.block_x), blk(L.block_x);
    const int key = (parity ? 4 : 0) + (ph.collision ? 2 : 0) + (ph.source == 2 ? 1 : 0);
    switch (key) {
#define SRC_CASE(P, C, SR)                                                                                    \
  case (P ? 4 : 0) + (C ? 2 : 0) + (SR == 2 ? 1 : 0):                                                          \
    hipLaunchKernelGGL((k_sweep<ST, D, MODEL, P, 0, C, false, false, false, SR>), grd, blk, 0, L.stream, g, ph, cd, \
                       Body{}, nullptr, nullptr, Inflow{}, MomentsOut{});                                        \
    break;
      SRC_CASE(0, 0, 1) SRC_CASE(0, 0, 2) SRC_CASE(0, 1, 1) SRC_CASE(0, 1, 2)
      SRC_CASE(1, 0, 1) SRC_CASE(1, 0, 2) SRC_CASE(1, 1, 1) SRC_CASE(1, 1, 2)
#undef SRC_CASE
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  } else {
    (void)L, (void)g, (void)ph, (void)cd, (void)parity;
    return hipErrorInvalidValue;
  }
}

// k_sweep2 serves FP16/BF16 storage of the 8-, 5- and 9-variable models (the 26-variable
// one's 182 packed words per lane do not fit the registers; the 13-component one's
// pair sweep needs about 300 VGPRs at parity 1, one wavefront per SIMD, and measured
// slower than its one-cell sweep: 3.7 against 4.5 TB/s) with the direct source, on
// periodic lattices, and D3Q7 ideal lattices with static faces (x faces in the sweep, y
// and z faces in the face pass) and a body -- the sweep outside the body's box, the box
// left to a one-cell sweep (mask_ok: the caller handles the bounce-back mask that way).
// Its workgroup width: the first of block_x, block_x / 2, block_x / 4 that is a multiple
// of 64 and whose 2 x width cells tile every x row; 0 if none does (the one-cell sweep
// runs).
inline int pair_width(const Grid& g, int block_x, bool faces, bool mask_ok = false) {
  if (g.mask && !mask_ok) return 0;
  for (int f = 0; f < 6; ++f)
    if (g.bc[f] && !faces) return 0;
  if (g.bc[0] && !fuse_x_faces(g)) return 0;
  for (int b = block_x, n = 0; n < 3 && b >= 64; b /= 2, ++n)
    if (b % 64 == 0 && g.nx % (2 * b) == 0) return b;
  return 0;
}

template <int ST, int D, int MODEL, bool BOX = false>
hipError_t sweep2_t(const Launch& L, const Grid& g, const Phys& ph, const Codec& cd, int parity, int bw,
                    const Body& b = Body{}, const Inflow& in = Inflow{}) {
  const dim3 grd((unsigned)((long long)(g.nx / (2 * bw)) * g.ny * g.nz)), blk((unsigned)bw);
  constexpr bool kF = D == 3 && MODEL == 0;  // x faces possible
  auto go = [&](auto par_c, auto coll_c, auto fx_c) {
    constexpr int P = decltype(par_c)::value, C = decltype(coll_c)::value;
    constexpr bool FXv = decltype(fx_c)::value;
    hipLaunchKernelGGL((k_sweep2<ST, D, MODEL, P, C, BOX, FXv>), grd, blk, 0, L.stream, g, ph, cd, b, in);
  };
  using I0 = std::integral_constant<int, 0>;
  using I1 = std::integral_constant<int, 1>;
  auto with_fx = [&](auto par_c, auto coll_c) {
    if constexpr (kF) {
      if (g.bc[0]) return go(par_c, coll_c, std::true_type{});
    }
    go(par_c, coll_c, std::false_type{});
  };
  auto with_coll = [&](auto par_c) {
    if (ph.collision) return with_fx(par_c, I1{});
    with_fx(par_c, I0{});
  };
  if (parity == 0)
    with_coll(I0{});
  else
    with_coll(I1{});
  return hipGetLastError();
}

template <int ST, int D, int MODEL>
hipError_t sweep_t(const Launch& L, const Grid& g, const Phys& ph, const Codec& cd, int parity, const Inflow& in) {
  if (ph.source != 0) return sweep_src_t<ST, D, MODEL>(L, g, ph, cd, parity);
  if constexpr ((ST == ST_F16 || ST == ST_BF16) && MODEL != 1 && MODEL != 4) {
    if (const int bw = pair_width(g, L.block_x, D == 3 && MODEL == 0))
      return sweep2_t<ST, D, MODEL>(L, g, ph, cd, parity, bw, Body{}, in);
  }
  launch_k<ST, D, MODEL, 0, false>(L, cell_grid(g, L.block_x), parity, ph.collision, lane_exchange(g, L.block_x, MODEL),
                                   fuse_x_faces(g), g, ph, cd, Body{}, nullptr, nullptr, in);
  return hipGetLastError();
}

template <int ST>
hipError_t sweep_inj_t(const Launch& L, const Grid& g, const Phys& ph, const Codec& cd, int parity,
                       const float* dq, const int* ctl, const MomentsOut& mo) {
  if (L.dim == 2)
    launch_k<ST, 2, 0, 0, true>(L, cell_grid(g, L.block_x), parity, 0, lane_exchange(g, L.block_x, 0), false, g, ph,
                                cd, Body{}, dq, ctl, Inflow{}, mo);
  else
    launch_k<ST, 3, 0, 0, true>(L, cell_grid(g, L.block_x), parity, 0, lane_exchange(g, L.block_x, 0), false, g, ph,
                                cd, Body{}, dq, ctl, Inflow{}, mo);
  return hipGetLastError();
}

// what 1: the bounce-back body; 3: the homogenized body
template <int ST>
hipError_t sweep_body_t(const Launch& L, const Grid& g, const Phys& ph, const Codec& cd, int parity,
                        const Body* b, int what, const Inflow& in) {
  const dim3 grd = cell_grid(g, L.block_x);
  const bool fx = fuse_x_faces(g);
  const int bx = b->box[1] - b->box[0], by = b->box[3] - b->box[2], bz = b->box[5] - b->box[4];
  if (what == 1) {
    // the plain sweep outside the body's box, which holds every solid cell and every cut
    // link (two cells per lane in FP16/BF16, else one with the lane exchange), and the
    // one-cell bounce-back sweep of the box; the two update disjoint cells.  The box must
    // keep clear of the x faces the outside sweep re-sets and of the cells next to them,
    // whose moments a zero-gradient face takes; else the bounce-back sweep takes every cell.
    if (b->box[0] > 1 && b->box[1] < g.nx - 1) {
      bool pair = false;
      if constexpr (ST == ST_F16 || ST == ST_BF16) {
        if (const int bw = pair_width(g, L.block_x, true, true)) {
          const hipError_t e = sweep2_t<ST, 3, 0, true>(L, g, ph, cd, parity, bw, *b, in);
          if (e != hipSuccess) return e;
          pair = true;
        }
      }
      if (!pair)
        launch_k<ST, 3, 0, 3, false>(L, grd, parity, ph.collision, lane_exchange(g, L.block_x, 0), fx, g, ph, cd, *b,
                                     nullptr, nullptr, in);
      if (bx > 0 && by > 0 && bz > 0) {
        const dim3 bgrd((unsigned)((bx + L.block_x - 1) / L.block_x), (unsigned)by, (unsigned)bz);
        launch_k<ST, 3, 0, 4, false>(L, bgrd, parity, ph.collision, false, false, g, ph, cd, *b, nullptr, nullptr, in);
      }
      return hipGetLastError();
    }
    launch_k<ST, 3, 0, 1, false>(L, grd, parity, ph.collision, false, fx, g, ph, cd, *b, nullptr, nullptr, in);
  } else {
    // homogenized body: the plain sweep outside the body's box, then the homogenized
    // sweep of the box; the two update disjoint cells, each cell exactly once
    bool pair = false;
    if constexpr (ST == ST_F16 || ST == ST_BF16) {
      if (const int bw = pair_width(g, L.block_x, true)) {
        const hipError_t e = sweep2_t<ST, 3, 0, true>(L, g, ph, cd, parity, bw, *b, in);
        if (e != hipSuccess) return e;
        pair = true;
      }
    }
    if (!pair)
      launch_k<ST, 3, 0, 3, false>(L, grd, parity, ph.collision, lane_exchange(g, L.block_x, 0), fx, g, ph, cd, *b,
                                   nullptr, nullptr, in);
    if (bx > 0 && by > 0 && bz > 0) {
      const dim3 bgrd((unsigned)((bx + L.block_x - 1) / L.block_x), (unsigned)by, (unsigned)bz);
      launch_k<ST, 3, 0, 2, false>(L, bgrd, parity, ph.collision, false, false, g, ph, cd, *b, nullptr, nullptr, in);
    }
  }
  return hipGetLastError();
}

template <int ST, int D, int M>
struct SweepFn {
  static hipError_t run(const Launch& L, const Grid& g, const Phys& ph, const Codec& cd, int par, const Inflow& in) {
    return sweep_t<ST, D, M>(L, g, ph, cd, par, in);
  }
};

}  // namespace

hipError_t launch_sweep(const Launch& L, const Grid& g, const Phys& ph, const Codec& cd, int parity,
                        const Inflow& in) {
  return dispatch<SweepFn>(L, g, ph, cd, parity, in);
}

hipError_t launch_sweep_inj(const Launch& L, const Grid& g, const Phys& ph, const Codec& cd, int parity,
                            const float* dq, const int* ctl, const MomentsOut& mo) {
  if ((L.dim != 2 && L.dim != 3) || L.model != 0 || ph.collision != 0) return hipErrorInvalidValue;
  if (L.dim == 3 && (g.bc[0] || g.bc[2] || g.bc[4] || g.mask)) return hipErrorInvalidValue;  // periodic, no body
  switch (L.storage) {
    case ST_F64: return sweep_inj_t<ST_F64>(L, g, ph, cd, parity, dq, ctl, mo);
    case ST_F32: return sweep_inj_t<ST_F32>(L, g, ph, cd, parity, dq, ctl, mo);
    case ST_F16: return sweep_inj_t<ST_F16>(L, g, ph, cd, parity, dq, ctl, mo);
    case ST_BF16: return sweep_inj_t<ST_BF16>(L, g, ph, cd, parity, dq, ctl, mo);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_sweep_body(const Launch& L, const Grid& g, const Phys& ph, const Codec& cd, int parity,
                             const Body& b, int mode, const Inflow& in) {
  if (L.dim != 3 || L.model != 0) return hipErrorInvalidValue;
  if (mode != 2 && (mode != 1 || !g.mask)) return hipErrorInvalidValue;
  const int what = mode == 2 ? 3 : 1;
  switch (L.storage) {
    case ST_F64: return sweep_body_t<ST_F64>(L, g, ph, cd, parity, &b, what, in);
    case ST_F32: return sweep_body_t<ST_F32>(L, g, ph, cd, parity, &b, what, in);
    case ST_F16: return sweep_body_t<ST_F16>(L, g, ph, cd, parity, &b, what, in);
    case ST_BF16: return sweep_body_t<ST_BF16>(L, g, ph, cd, parity, &b, what, in);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace vlbm

// Internal interface between the C ABI (vlbm_api.hip) and the kernels (vlbm_sweep.hip,
// vlbm_kernels.hip).  Not installed; the public ABI is include/vlbm.h.
#pragma once

#include <hip/hip_runtime.h>

#include "vlbm_physics.h"

namespace vlbm {

enum Storage { ST_F64 = 0, ST_F32 = 1, ST_F16 = 2, ST_BF16 = 3 };

// Everything a sweep-family kernel needs, passed by value (kernel arguments).
struct Grid {
  void* f;              // population buffer, planes (k*NQ + i) of `stride` elements
  long long stride;     // elements per plane
  int nx, ny, nz;
  int bc[6];            // per face: 0 periodic, 1 inflow, 2 zero gradient
  unsigned char* mask;  // body mask per cell (NULL: no body), bits below
  void* sprev;          // Chai source operator: the previous step's source [K][N] in the
                        // compute type (double for FP64 storage, else float); else NULL
  int xf_pass = 0;      // 1: this step the face pass re-sets the x faces too (fuse_x_faces)
  int pk = 0;           // 1: variable pairs packed (16-bit storage of the 26-variable model):
                        // variables 2p and 2p + 1 of one slot share the 32-bit element of
                        // plane (p*Q + slot) -- `stride` words per plane, low half 2p
};

// 16-bit element index of population (variable k, slot, cell): planes (k*Q + slot) of
// `stride` elements, or with packed pairs planes (k/2*Q + slot) of `stride` 32-bit words.
__host__ __device__ inline size_t pop_index(const Grid& g, int nq, int k, int slot, unsigned cell) {
  return g.pk ? ((size_t)((k >> 1) * nq + slot) * (size_t)g.stride + cell) * 2 + (k & 1)
              : (size_t)(k * nq + slot) * (size_t)g.stride + cell;
}

// Body mask bits: solid now, solid before the last move, and for i = 1..6 the
// neighbour x + e_i is solid now (the link i is cut).
constexpr unsigned kSolid = 0x80u, kWasSolid = 0x01u;
__host__ __device__ constexpr unsigned link_bit(int i) { return 1u << i; }

// Moving rough sphere with a dipole field (absolute cell coordinates, time in steps).
struct Body {
  double c0[3], v[3], R0;
  double a[4], d[4][3], b[4], e[4][3];
  double m[3];
  double rmax;  // bound of the surface radius (cells)
  double t;     // time of the state the kernel works on
  int box[6];   // [x0, x1) x [y0, y1) x [z0, z1): the cells whose mask can change
};

// Boundary state of inflow faces (the first 8 conserved variables).
struct Inflow {
  double q[8];
};

// Optional outputs of the injecting sweep (learned correction): the pre-collision
// moments of every cell after the injection, FP32 [8][N] in x, and the network's
// standardised input, BF16 channels-last [N][8] in act ((x - mean[k]) * istd[k],
// rounded to nearest even).  x == NULL: none.
struct MomentsOut {
  float* x;
  unsigned short* act;
  const float* mean;
  const float* istd;
};

// FP16/BF16 deviation codec: f = rest[k*NQ+i] + sc[k*NQ+i] * h,
// h = round((f - rest) * isc).  Index i is the population's direction.
struct Codec {
  float rest[KMAX * 7];
  float sc[KMAX * 7];
  float isc[KMAX * 7];
};

struct Launch {
  int storage, dim, model;
  int block_x;
  hipStream_t stream;
};

// One sweep (collide + stream) at the given parity (0: natural layout in, swapped
// out; 1: swapped in, natural out).
hipError_t launch_sweep(const Launch& L, const Grid& g, const Phys& ph, const Codec& cd, int parity,
                        const Inflow& in);

// Static faces (D3Q7 ideal model): every node of a non-periodic face takes
// f := f^eq(Q_bc) at the given parity, Q_bc the inflow state on inflow faces, else
// the moments of the nearest cell that lies on no non-periodic face.
hipError_t launch_faces(const Launch& L, const Grid& g, const Phys& ph, const Codec& cd, int parity,
                        const Inflow& in);

// The sweep itself re-sets the nodes of non-periodic x faces that lie on no other
// non-periodic face (D3Q7 ideal); it takes the zero-gradient state from the
// neighbouring lane, which holds cell x = 1 (x = nx - 2) unless nx - 1 starts a new
// wavefront.  The face pass then handles the y and z faces only.  A step whose body box
// reaches x <= 1 or x >= nx - 2 sets xf_pass: the cells of the box skip the outside
// sweep and the box sweep re-sets no face, so the face pass takes the x faces as well.
__host__ __device__ inline bool fuse_x_faces(const Grid& g) {
  return g.bc[0] != 0 && g.nx % 64 != 1 && !g.xf_pass;
}

// Body mask in b.box at time b.t: pass 0 sets the solid bit (and keeps the old one
// as kWasSolid unless `fresh`), pass 1 the link bits.
hipError_t launch_mask(const Launch& L, const Grid& g, const Body& b, int pass, int fresh);
// Cells of b.box uncovered by the last move take f^eq of the mean moments of their
// neighbours that are fluid before and after it (the inflow state if none), at the
// given parity.
hipError_t launch_refill(const Launch& L, const Grid& g, const Phys& ph, const Codec& cd, int parity,
                         const Body& b, const Inflow& in);
// Sweep of a D3Q7 ideal lattice with a body at time b.t.  mode 1: solid cells are
// skipped and links into the body bounce back (moving wall, dipole field); mode 2:
// every cell collides toward its homogenized state (porosity blending).
hipError_t launch_sweep_body(const Launch& L, const Grid& g, const Phys& ph, const Codec& cd, int parity,
                             const Body& b, int mode, const Inflow& in);

// Control block of a pending learned correction (device, 32-bit words): ctl[0] nonzero
// means "add it"; ctl[1 + 8 b + k] holds, as an FP32 bit pattern, the mean that channel k
// of lattice b loses (its projection onto zero lattice totals; 0 without projection).
// Lattice b is the slice z for a batch of 2D lattices and 0 for a 3D lattice.  The
// correction added is w_i (dq[k][c] - mean[b][k]), the difference taken in FP32.
__host__ __device__ inline int inj_lattice(int dim, int z) { return dim == 2 ? z : 0; }

// Sweep of a periodic 2D or 3D ideal-MHD BGK lattice (any storage form) that first
// adds the pending correction of control block ctl (above) to the gathered, decoded
// populations (dq FP32 [K][N], device).
hipError_t launch_sweep_inj(const Launch& L, const Grid& g, const Phys& ph, const Codec& cd, int parity,
                            const float* dq, const int* ctl, const MomentsOut& mo);

// The learned correction's network input from the populations at the given parity
// (8-variable ideal model): the moments of every cell, FP32 in mo.x, and their
// standardised BF16 form in mo.act (as MomentsOut describes).
hipError_t launch_net_input(const Launch& L, const Grid& g, const Codec& cd, int parity, const MomentsOut& mo);

// f := f^eq(Q) in natural layout.  Q is device SoA [K][N], FP64 or FP32.
hipError_t launch_init(const Launch& L, const Grid& g, const Phys& ph, const Codec& cd,
                       const void* Q, int q_is_f32);

// Moments at the given parity: Qout [K][N] FP64 (device), per-block partial sums
// [nblk][K+5] (sum Q_k, sum d, sum d^2, max |d|, unused, bad count).
hipError_t launch_moments(const Launch& L, const Grid& g, const Phys& ph, const Codec& cd,
                          int parity, double* Qout, double* partial, int nblk);
// Central div B of the moment field: per-block partial sums of its square [nblk].
hipError_t launch_divc(const Launch& L, const Grid& g, const double* Qout, double* partial,
                       int nblk);
// Fixed-order reduction of per-block partials [nblk][n] into out[n] (device);
// slots whose bit is set in maxmask take the max, the others the sum.
// Loads on the homogenized body at time b.t over b.box: nblk block partials of
// (force[3], torque[3], energy, magnetic flux), to be summed with launch_reduce.
hipError_t launch_body_loads(const Launch& L, const Grid& g, const Phys& ph, const Codec& cd, int parity,
                             const Body& b, double* partial, int nblk);
hipError_t launch_reduce(const Launch& L, int n, const double* partial, int nblk, unsigned maxmask,
                         double* out);

// Decoded populations at listed cells: out[n][K][NQ] FP64.
hipError_t launch_gather(const Launch& L, const Grid& g, const Codec& cd, int parity, int K,
                         const long long* cells, long long n, double* out);

// Per-variable sum (mode 0) or max |Q_k - rest_k| (mode 1) over a device field
// Q [K][N] (FP64 or FP32); result out[K] FP64 (device).
hipError_t launch_field_reduce(const Launch& L, long long N, int K, const void* Q, int q_is_f32,
                               int mode, const double* rest, double* partial, int nblk, double* out);

// FP64 -> FP32 conversion of n values.
hipError_t launch_to_f32(hipStream_t s, const double* in, float* out, long long n);

// Streaming 16-byte copy.
hipError_t launch_copy(hipStream_t s, void* dst, const void* src, size_t bytes);

}  // namespace vlbm

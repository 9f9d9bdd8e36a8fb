// Internal interface between the C ABI (vlbm_api.hip) and the kernels
// (vlbm_kernels.hip).  Not installed; the public ABI is include/vlbm.h.
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
  int bc[6];            // per face: 0 periodic (only kind handled by the periodic sweep)
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
hipError_t launch_sweep(const Launch& L, const Grid& g, const Phys& ph, const Codec& cd, int parity);

// Sweep of a 2D ideal-MHD lattice (FP32 or FP64 storage) that first adds
// *flag * w_i dq[k][c] to the gathered populations (dq FP32 [K][N], device).
hipError_t launch_sweep_inj(const Launch& L, const Grid& g, const Phys& ph, const Codec& cd, int parity,
                            const float* dq, const int* flag);

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

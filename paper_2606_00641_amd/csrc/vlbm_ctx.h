// Internal: the context behind the opaque vlbm_ctx handle (shared by the C ABI of
// the sweep and of the learned correction).  Not installed.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "vlbm.h"
#include "vlbm_kernels.h"

struct vlbm_ctx {
  vlbm_params p{};
  int D = 0, K = 0, NQ = 0, esize = 0;
  long long N = 0, stride = 0;
  size_t pop_bytes = 0;
  void* f = nullptr;
  bool owned = false;
  hipStream_t stream = nullptr;
  int device = 0;                 // the device current at vlbm_create
  vlbm::Phys ph{};
  vlbm::Codec cd{};
  vlbm::Grid g{};
  vlbm::Launch L{};
  double rest_Q[vlbm::KMAX] = {};
  double scale[vlbm::KMAX] = {};
  bool rest_given = false;
  int nblk = 0;
  double* d_partial = nullptr;   // [nblk][K+5]
  double* d_partial2 = nullptr;  // [nblk]
  double* d_totals = nullptr;    // [K+5] totals, then 2 x KMAX codec scratch
  double* d_Q = nullptr;         // [K][N] moments scratch (lazy)
  bool has_faces = false;         // some face is not periodic
  vlbm::Inflow inflow{};
  vlbm::Body body{};              // geometry; t and box set per launch
  double body_rmax = 0.0;         // bound of the body's surface radius
  unsigned char* d_mask = nullptr;  // [N] body mask (body only)
  void* d_sprev = nullptr;          // [K][N] previous-step source (Chai's source operator only)
  long long step = 0;
  // identity of this context (unique in the process) and the generation of what kernel
  // launches take by value (the codec changes at init and restore); a graph captured
  // from this context is valid while both are unchanged
  long long uid = 0, gen = 0;
  bool initialized = false;
  std::string err;
};

// One step of an initialised context on its stream (vlbm_step's body): static faces,
// the sweep (with the body and its move), step + 1.  Errors are recorded in c->err.
vlbm_status vlbm_step_one(vlbm_ctx* c);

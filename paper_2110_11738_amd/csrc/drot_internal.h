// Internal declarations shared by the kernel and host translation units of
// libdrot.so.  Not part of the public ABI (see include/drot.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace drot {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kWaves = 4;          // waves per sweep workgroup
constexpr int kBlock = kWave * kWaves;
constexpr int kAuxBlock = 256;     // threads per aux workgroup
constexpr int kTileSlots = 4;      // per-tile scalar partials (see TileSlot)
constexpr int kAuxSlots = 13;      // per-aux-block scalar partials (see AuxSlot)
constexpr int kTraceCap = 65536;   // per-iteration records kept on the device
constexpr int kTraceWidth = 8;

// What one sweep launch does.
enum SweepMode : int {
  kIter = 0,    // Algorithm 1 step 4 + the sums of step 5, <C,X>, r_dual partial
  kInitPQ = 1,  // write X_0 = p q^T; its row/column sums; |C|_F^2; finiteness
  kInitX = 2,   // X_0 given: its row/column sums; |C|_F^2; finiteness
  kFinal = 3,   // read-only FP64 evaluation of (X, phi, psi)
};

enum TileSlot : int { kTsCost = 0, kTsDual = 1, kTsCsq = 2, kTsBad = 3 };

enum AuxSlot : int {
  kAsR = 0,     // sum r_i            (rows)
  kAsR2,        // sum r_i^2
  kAsPphi,      // sum p_i * phi_i    (phi without its scalar part, except kFinal)
  kAsS,         // sum s_j            (columns)
  kAsS2,        // sum s_j^2
  kAsQpsi,      // sum q_j * psi_j
  kAsT0,        // tile slot kTsCost (or kTsCsq in init), reduced over a tile range
  kAsT1,        // tile slot kTsDual (or kTsBad in init)
  kAsP,         // init: sum p, later unused
  kAsQ,         // init: sum q
  kAsP2,        // init: sum p^2 + sum q^2
  kAsNeg,       // init: count of negative marginal entries
  kAsNonfin,    // init: count of non-finite marginal / warm-start entries
};

// Scalars of the iteration, resident on the device.  The host writes the
// problem block at bind time and reads the whole record when polling.
struct DevState {
  // --- problem (host-written at bind) ---
  double rho, tol;
  int64_t max_iter;
  int32_t tol_mode, pad0;
  int64_t m, n;
  // --- filled by the initialisation pass ---
  double sum_p, sum_q, norm_pq, norm_c;
  double sum_phi0, sum_psi0;
  double init_bad;          // count of non-finite entries (C, X_0, p, q, warm start), negative X_0
  double init_neg;          // count of negative marginal entries
  // --- iteration ---
  double alpha;             // alpha_k
  double cphi, cpsi;        // scalar parts of phi_k and psi_k: (2 beta - alpha)/n, /m
  int64_t iter;             // iterations completed
  int32_t done, status;     // stop flag; 0 converged, 1 max_iter, -3 non-finite
  int64_t stop_iter;
  uint64_t t_start, t_stop; // wall_clock64 ticks: initialisation start, stop
  uint64_t t_last;          // end of the latest iteration
  double pobj, dobj, rp, rd, gap, test;
  // --- final evaluation ---
  double f_pobj, f_dobj, f_rp, f_rd, f_gap, f_eps_p, f_eps_d, f_eps_g;
  // --- aux completion counter (last workgroup finishes the scalars) ---
  uint32_t counter, pad1;
};

// Geometry of one sweep launch.
struct SweepGeom {
  int64_t m, n;
  int64_t ldc, ldx;
  int n_ct;         // column tiles
  int n_rb;         // row blocks
  int rows;         // rows per workgroup tile
};

struct SweepArgs {
  const void* C;
  void* X;
  const void* p;           // typed like X (init only)
  const void* q;
  const void* phiT;        // typed like X: phi without its scalar part
  const void* psiT;
  const double* phi64;     // final pass: phi without its scalar part (FP64)
  const double* psi64;
  DevState* st;
  void* colpart;           // [n_rb][n]  (float in the FP32 iteration, else double)
  void* rowpart;           // [n_ct][m]
  double* tiles;           // [n_tiles][kTileSlots]
  SweepGeom g;
};

struct AuxArgs {
  const void* p;           // typed like X
  const void* q;
  const void* colpart;
  const void* rowpart;
  const double* tiles;
  double* a;               // [m]
  double* b;               // [n]
  double* phi64;           // [m]
  double* psi64;           // [n]
  void* phiT;              // [m] typed like X
  void* psiT;              // [n]
  const double* mu0;       // warm start (init only), may be null
  const double* nu0;
  double* mu_out;          // final only, may be null
  double* nu_out;
  double* blockpart;       // [nblocks][kAuxSlots]
  double* trace;           // [kTraceCap][kTraceWidth]
  DevState* st;
  int64_t m, n;
  int n_ct, n_rb;          // producers of rowpart / colpart
  int n_tiles;
  int row_blocks, col_blocks;
  double wall_rate;        // wall_clock64 ticks per second
};

// Launchers (drot_kernels.hip).  `vec` is 4 (float) / 2 (double) for 16-byte
// loads or 1 for the scalar fallback; `chunks` the chunks per lane.
hipError_t launch_sweep(int dtype, int mode, int vec, int chunks, const SweepArgs& a,
                        hipStream_t s);
hipError_t launch_aux(int dtype, int mode, const AuxArgs& a, hipStream_t s);
hipError_t launch_prep(const AuxArgs& a, hipStream_t s);

}  // namespace drot

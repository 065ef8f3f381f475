// Internal declarations shared by the kernel and host translation units of
// libdrot.so.  Not part of the public ABI (see include/drot.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace drot {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kWaves = 4;          // waves per sweep workgroup
constexpr int kBlock = kWave * kWaves;
constexpr int kTileSlots = 2;      // per-tile scalar partials (see TileSlot)
constexpr int kSlots = 13;         // per-finisher scalar partials (see Slot)
constexpr int kTraceCap = 65536;   // per-iteration records kept on the device
constexpr int kTraceWidth = 8;
constexpr int kAuxCols = 64;       // columns per aux column workgroup
constexpr int kAuxRows = kWave;    // rows per aux row workgroup
constexpr int kAuxSplitMin = 256;  // from this many aux workgroups: separate finishing launch
// One-workgroup iteration for small problems (see small_kernel).
// One-workgroup path: kSmallBlock threads (16 waves) hold the plan and the
// cost in registers, small_slots(dtype) entries of each per thread: wave w
// owns rows w, w + 16, ... (small_rows of them), lane l the columns
// l, l + 64, ... (small_cols of them, a power of two up to 8).
constexpr int kSmallBlock = 1024;
constexpr int kSmallWaves = kSmallBlock / kWave;
constexpr int small_slots(int dtype) { return dtype == 0 ? 32 : 16; }
constexpr int small_cols(int64_t n) {
  return n <= kWave ? 1 : n <= 2 * kWave ? 2 : n <= 4 * kWave ? 4 : n <= 8 * kWave ? 8 : 0;
}
constexpr bool small_fits(int dtype, int64_t m, int64_t n) {
  return m >= 1 && n >= 1 && small_cols(n) > 0 &&
         m <= (int64_t)kSmallWaves * (small_slots(dtype) / small_cols(n));
}

// Workgroups of one aux launch: column groups of kAuxCols, then row groups of
// kAuxRows.
__host__ __device__ inline int64_t aux_workgroups(int64_t m, int64_t n) {
  return (n + kAuxCols - 1) / kAuxCols + (m + kAuxRows - 1) / kAuxRows;
}

// What one sweep + aux pair does.
enum SweepMode : int {
  kIter = 0,    // Algorithm 1 steps 4-8 and the stopping test
  kInitPQ = 1,  // steps 1-2 with X_0 = p q^T written; |C|_F; finiteness checks
  kInitX = 2,   // steps 1-2 with X_0 given (read only)
  kFinal = 3,   // read-only FP64 evaluation of (X, phi, psi); writes mu, nu
  // The paper's skip-C schedule (Claim 1): iterations alternate between
  kIterA = 4,   // reads X and C, stores W = X_{k+1} - rho C (stopping test as kIter)
  kIterB = 5,   // reads W only: X_{k+2} = [W + phi e^T + f psi^T]_+ (no test)
  kFinalW = 6,  // restores X = W + rho C and evaluates like kFinal
};

// Where the sweep takes c_ij from.
enum CostKind : int {
  kCostDense = 0,   // C stored densely in the problem type
  kCostBF16 = 1,    // C stored densely as bfloat16 (float32 problems)
  kCostCoords = 2,  // c_ij = scale * |xs_i - xt_j|^2 from float32 coordinates
};

// Per-tile scalars: iteration/final: <C,X> and sum [t]_+^2; init: |C|^2 and
// the count of non-finite entries.
enum TileSlot : int { kTs0 = 0, kTs1 = 1 };

enum Slot : int {
  kSR = 0,      // sum r_i  (init: sum a_i)
  kSR2,         // sum r_i^2
  kSPphi,       // sum p_i phi_i (phi without its scalar part, except in kFinal)
  kSS,          // sum s_j  (init: sum b_j)
  kSS2,         // sum s_j^2
  kSQpsi,       // sum q_j psi_j
  kST0,         // tile slot kTs0 summed over a slice of tiles
  kST1,         // tile slot kTs1
  kSP,          // init: sum p
  kSQ,          // init: sum q
  kSPQ2,        // init: sum p^2 + sum q^2
  kSNeg,        // init: count of negative marginal entries
  kSNonfin,     // init: count of non-finite marginal / warm-start entries
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
  double cscale;            // coordinates cost: scale (host-given, or 1 / max from maxc)
  uint32_t maxc_bits;       // coordinates cost: bit pattern of max |xs_i - xt_j|^2 (float)
  uint32_t pad2;
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
  // --- completion counter of the finishers (the last one does the scalars) ---
  uint32_t counter, pad1;
};

// Geometry of one sweep launch.
struct SweepGeom {
  int64_t m, n;
  int64_t ldc, ldx;
  int64_t ldcp;     // row stride of colpart (n rounded up to a multiple of 4)
  int n_ct;         // column strips
  int n_rb;         // row blocks of `rows` rows
  int n_rg;         // row groups: workgroup (strip, g) sweeps row blocks g, g + n_rg, ...
  int rows;         // rows per row block
};

struct SweepArgs {
  int cost_kind;           // CostKind
  int dim;                 // coordinates cost: point dimension
  const float* xs;         // coordinates cost: m x dim
  const float* xt;         // coordinates cost: n x dim
  const void* C;           // dense cost (problem type) or bfloat16 bit patterns
  void* X;
  const void* p;           // typed like X
  const void* q;
  void* phiT;              // [m] typed like X: phi without its scalar part
  void* psiT;              // [n]
  double* phi64;           // [m] the same in FP64
  double* psi64;           // [n]
  double* a;               // [m] accumulator a_k
  double* b;               // [n] accumulator b_k
  const double* mu0;       // warm start (init only), may be null
  const double* nu0;
  double* mu_out;          // final only, may be null
  double* nu_out;
  DevState* st;
  void* colpart;           // [n_rg][ldcp] (float in the FP32 iteration, else double)
  void* rowpart;           // [n_ct][m]
  double* tiles;           // [n_rg * n_ct][kTileSlots], workgroup (g, ct) at g * n_ct + ct
  double* blockpart;       // [kSlots][aux workgroups] (slot-major)
  // Pending form of the iteration (few aux workgroups; see drot_kernels.hip):
  // the scalar steps that close the previous iteration run at the start of
  // the sweep, from that iteration's state record `st_prev` and the aux sums
  // `bp_prev`; workgroup 0 commits the result to `st`.  nullptr: `st`
  // already holds the state entering the iteration.  A one-wave finishing
  // launch reads the same pair (st_prev, bp_prev) and commits into `st`.
  const DevState* st_prev;
  const double* bp_prev;
  int prev_b;              // the previous iteration was a C-free (kIterB) one
  double* trace;           // [trace_cap][kTraceWidth]
  int64_t trace_cap;       // records kept (ring)
  double wall_rate;        // wall_clock64 ticks per second
  SweepGeom g;
};

// Tile variant of the sweep: `vec` is 4 (float) / 2 (double) for 16-byte
// loads or 1 for the scalar fallback; `chunks` the chunks per lane (1/2, or
// 1/4 on the scalar path); `unroll` the rows kept in flight (4 or 8);
// `stream` selects nontemporal loads and stores.  Ragged widths use 4 rows in
// flight.
struct TileCfg {
  int vec, chunks, unroll;
  bool stream;
  bool ragged;      // 16-byte path with n not a multiple of vec (masked last chunk)
  bool comp = false;  // compensated per-lane sums, float64 partials (float32 iteration)
};

// Launchers (drot_kernels.hip).
// With e0 / e1 given, the sweep goes through hipExtLaunchKernel, which
// records the dispatch's own start and end times in those events.
hipError_t launch_sweep(int dtype, int mode, const TileCfg& t, const SweepArgs& a,
                        hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// `wide`: the float32 iteration's partials are float64 (compensated sweep).
// `publish`: the aux workgroups only publish their sums (pending form of the
// iteration); the scalar steps run in the next sweep or in launch_finish.
hipError_t launch_aux(int dtype, int mode, const SweepArgs& a, hipStream_t s, bool wide = false,
                      bool publish = false);
// One wave: the scalar steps of an iteration of mode `mode` from
// (a.st_prev, a.bp_prev), committed to a.st.
hipError_t launch_finish(int mode, const SweepArgs& a, hipStream_t s);
hipError_t launch_prep(const SweepArgs& a, hipStream_t s);
// `iters` iterations of a small problem in one one-workgroup launch.
hipError_t launch_small(int dtype, const SweepArgs& a, int64_t iters, hipStream_t s);
hipError_t launch_maxc(const SweepArgs& a, hipStream_t s);

// Batched problems: `args` (device) holds one SweepArgs per problem; the work
// lists hold (problem, workgroup) pairs for the sweep and the aux kernel of
// one iteration (dense cost, 4 rows in flight).
hipError_t launch_batch_step(int dtype, int mode, const TileCfg& t, const SweepArgs* args,
                             const uint2* sweep_work, int64_t n_sweep, const uint2* aux_work,
                             int64_t n_aux, int n_prob, hipStream_t s);
hipError_t launch_prep_batch(const SweepArgs* args, int count, hipStream_t s);

}  // namespace drot

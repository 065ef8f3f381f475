// HIP kernels of the DROT hot path for gfx950 (CDNA4, wave64).
//
// One iteration of Algorithm 1 (DROT) is two launches:
//
//  sweep_kernel  one fused pass over the dense m x n plan.  Each entry is read
//                once (X and C) and written once (X):
//                    t     = phi_i + psi_j - rho c_ij
//                    x_ij <- max(x_ij + t, 0)                       (step 4)
//                and in the same pass the kernel accumulates row sums, column
//                sums (step 5), <C, X_{k+1}> and sum [t]_+^2 = rho^2 r_dual^2
//                at the incoming shifts (Section 3, stopping criteria), and
//                writes them as per-tile partials.
//  aux_kernel    the O(m+n) part: level-2 sums of the partials in a fixed
//                order; r = u - p, s = v - q; the vector parts of the new
//                shifts phi~ = (a - 2r)/n, psi~ = (b - 2s)/m; a <- a - r,
//                b <- b - s (steps 5-8).  The last workgroup to finish sums
//                the workgroups' scalar partials in a fixed order and does the
//                scalar steps: beta = f^T r/(m+n), the common scalar part
//                (2 beta - alpha) of the new shifts, alpha <- alpha - beta,
//                and the stopping test.  With many aux workgroups (and in the
//                batched solver) a separate one-wave finish_kernel does these
//                scalar steps instead, after the aux launch.
//
// The shifts are kept as phi = phi~ + (2 beta - alpha)/n and
// psi = psi~ + (2 beta - alpha)/m (the algebra of steps 6-7): the vector parts
// need no global quantity, and the next sweep adds the two scalar parts to its
// row shift, so no second pass over the vectors is needed once beta is known.
//
// Every sum runs in a fixed order, so results are bit-reproducible; the only
// atomics are the integer counter that elects the last aux workgroup and the
// maximum of the coordinates cost (order-independent).
//
// Differences from the paper's CUDA kernel (Section 3, "Main kernel"): that
// kernel is column-major with one thread per row and sums columns with float
// atomics.  Here X is row-major, the 64 lanes of a wavefront run along a row
// with 16-byte loads, each lane keeps the column partials of its columns in
// registers over the tile's rows, row sums use DPP cross-lane reductions, and
// column partials go through a deterministic two-level tree.  The kernel
// boundary between sweep and aux is the device-wide release/acquire point: a
// device-scope fence inside the sweep would write back the L2 (full of the
// freshly written plan) once per workgroup.
#include <hip/hip_ext.h>
#include <type_traits>

#include "drot_internal.h"

namespace drot {
namespace {

// ---------------------------------------------------------------------------
// Wave-level sum with DPP (all 64 lanes active).  Fixed combination order;
// the result is read from lane 63.
// ---------------------------------------------------------------------------
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, ROW_MASK, 0xf, false);
}

template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp(float v) {
  return __builtin_bit_cast(float, dpp_i<CTRL, ROW_MASK>(__builtin_bit_cast(int, v)));
}

template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ double dpp(double v) {
  const unsigned long long bits = __builtin_bit_cast(unsigned long long, v);
  const int lo = dpp_i<CTRL, ROW_MASK>((int)(unsigned)(bits & 0xffffffffull));
  const int hi = dpp_i<CTRL, ROW_MASK>((int)(unsigned)(bits >> 32));
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ float lane63(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}

__device__ __forceinline__ double lane63(double v) {
  const unsigned long long bits = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = __builtin_amdgcn_readlane((int)(unsigned)(bits & 0xffffffffull), 63);
  const unsigned hi = __builtin_amdgcn_readlane((int)(unsigned)(bits >> 32), 63);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

template <typename V>
__device__ __forceinline__ V wave_sum(V v) {
  v += dpp<0xB1>(v);         // quad_perm [1,0,3,2]: pairs
  v += dpp<0x4E>(v);         // quad_perm [2,3,0,1]: quads
  v += dpp<0x141>(v);        // row_half_mirror: groups of 8
  v += dpp<0x140>(v);        // row_mirror: rows of 16
  v += dpp<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
  v += dpp<0x143, 0xC>(v);   // row_bcast:31 into rows 2 and 3
  return lane63(v);
}

// wave_sum of N values at once: each DPP step is applied to all N before the
// next, so that the N dependency chains overlap.  Every lane gets the totals.
template <int N>
__device__ __forceinline__ void wave_sum_n(double (&v)[N]) {
#pragma unroll
  for (int s = 0; s < N; ++s) v[s] += dpp<0xB1>(v[s]);
#pragma unroll
  for (int s = 0; s < N; ++s) v[s] += dpp<0x4E>(v[s]);
#pragma unroll
  for (int s = 0; s < N; ++s) v[s] += dpp<0x141>(v[s]);
#pragma unroll
  for (int s = 0; s < N; ++s) v[s] += dpp<0x140>(v[s]);
#pragma unroll
  for (int s = 0; s < N; ++s) v[s] += dpp<0x142, 0xA>(v[s]);
#pragma unroll
  for (int s = 0; s < N; ++s) v[s] += dpp<0x143, 0xC>(v[s]);
#pragma unroll
  for (int s = 0; s < N; ++s) v[s] = lane63(v[s]);
}

// ---------------------------------------------------------------------------
// Types and memory helpers.
// ---------------------------------------------------------------------------
// Partial sums of the float32 iteration are float32 (per tile); everything
// else accumulates in float64.
constexpr bool is_iter(int mode) { return mode == kIter || mode == kIterA || mode == kIterB; }
constexpr bool is_final(int mode) { return mode == kFinal || mode == kFinalW; }

template <typename T, int MODE>
struct PartialOf {
  using type = typename std::conditional<std::is_same<T, float>::value && is_iter(MODE), float,
                                         double>::type;
};

// rho * c rounded once (never fused into a neighbouring add), so that the
// skip-C schedule's W = X - rho C and its restoration X = W + rho C use the
// same product and zero entries come back exactly zero.
template <typename A>
__device__ __forceinline__ A mul_rounded(A a, A b) {
#pragma clang fp contract(off)
  return a * b;
}

template <typename T, int VEC>
struct VecOf;
template <>
struct VecOf<float, 4> {
  typedef float type __attribute__((ext_vector_type(4)));
};
template <>
struct VecOf<double, 2> {
  typedef double type __attribute__((ext_vector_type(2)));
};

// 16-byte (or scalar) loads and stores; NT selects the nontemporal
// (streaming) cache policy, used when the plan and the cost matrix do not fit
// in the last-level cache.
template <typename T, int VEC, bool NT>
__device__ __forceinline__ void load_chunk(const T* ptr, T (&out)[VEC]) {
  if constexpr (VEC == 1) {
    out[0] = NT ? __builtin_nontemporal_load(ptr) : *ptr;
  } else {
    using V = typename VecOf<T, VEC>::type;
    const V* vp = reinterpret_cast<const V*>(ptr);
    const V v = NT ? __builtin_nontemporal_load(vp) : *vp;
#pragma unroll
    for (int e = 0; e < VEC; ++e) out[e] = v[e];
  }
}

template <typename T, int VEC, bool NT>
__device__ __forceinline__ void store_chunk(T* ptr, const T (&in)[VEC]) {
  if constexpr (VEC == 1) {
    if (NT) __builtin_nontemporal_store(in[0], ptr);
    else *ptr = in[0];
  } else {
    using V = typename VecOf<T, VEC>::type;
    V v;
#pragma unroll
    for (int e = 0; e < VEC; ++e) v[e] = in[e];
    if (NT) __builtin_nontemporal_store(v, reinterpret_cast<V*>(ptr));
    else *reinterpret_cast<V*>(ptr) = v;
  }
}

// VEC bfloat16 values (raw 16-bit patterns) widened exactly to float.
template <int VEC, bool NT>
__device__ __forceinline__ void load_bf16(const uint16_t* ptr, float (&out)[VEC]) {
  if constexpr (VEC == 1) {
    const uint16_t b = NT ? __builtin_nontemporal_load(ptr) : *ptr;
    out[0] = __builtin_bit_cast(float, (uint32_t)b << 16);
  } else {
    static_assert(VEC == 4, "bfloat16 chunks are 4 wide");
    typedef uint32_t u2 __attribute__((ext_vector_type(2)));
    const u2* vp = reinterpret_cast<const u2*>(ptr);
    const u2 v = NT ? __builtin_nontemporal_load(vp) : *vp;
    out[0] = __builtin_bit_cast(float, v[0] << 16);
    out[1] = __builtin_bit_cast(float, v[0] & 0xffff0000u);
    out[2] = __builtin_bit_cast(float, v[1] << 16);
    out[3] = __builtin_bit_cast(float, v[1] & 0xffff0000u);
  }
}

__device__ __forceinline__ bool finite_d(double v) { return __builtin_isfinite(v); }

__device__ __forceinline__ void store_agent(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double load_agent(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Block-wide fixed-order sum of kSlots values; result valid in thread 0.
__device__ __forceinline__ void block_sum_slots(double (&acc)[kSlots],
                                                double (&red)[kSlots][kWaves]) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  __syncthreads();  // `red` may still be read from a previous use
#pragma unroll
  for (int s = 0; s < kSlots; ++s) {
    const double v = wave_sum(acc[s]);
    if (lane == 0) red[s][wave] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int s = 0; s < kSlots; ++s) {
      double v = red[s][0];
#pragma unroll
      for (int w = 1; w < kWaves; ++w) v += red[s][w];
      acc[s] = v;
    }
  }
}

// The state scalars that the aux kernel and its finisher read.  Every
// workgroup loads them when it starts, so that the last workgroup's scalar
// steps wait on no further load; nothing in them changes during the launch
// (only the last workgroup writes the state, after all others are done).
// The value of one of two pointers, chosen by a wave-uniform condition.
// Each candidate is passed through readfirstlane first, so that the choice is
// made between values held in registers, never between addresses of
// argument fields (which would force the arguments into scratch memory).
template <typename P>
__device__ __forceinline__ P* pick(bool c, P* x, P* y) {
  auto uni = [](P* v) {
    const uint64_t u = reinterpret_cast<uint64_t>(v);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return reinterpret_cast<P*>(((uint64_t)hi << 32) | lo);
  };
  const P* px = uni(x);
  const P* py = uni(y);
  return const_cast<P*>(c ? px : py);
}

struct StateIn {
  double rho, tol, alpha, sum_p, sum_q, norm_pq, norm_c;
  double cphi, cpsi, sum_phi0, sum_psi0;
  int64_t iter, max_iter;
  uint64_t t_start;
  int tol_mode, done;
};

__device__ __forceinline__ StateIn load_state(const DevState* st) {
  StateIn v;
  v.rho = st->rho;
  v.tol = st->tol;
  v.alpha = st->alpha;
  v.sum_p = st->sum_p;
  v.sum_q = st->sum_q;
  v.norm_pq = st->norm_pq;
  v.norm_c = st->norm_c;
  v.cphi = st->cphi;
  v.cpsi = st->cpsi;
  v.sum_phi0 = st->sum_phi0;
  v.sum_psi0 = st->sum_psi0;
  v.iter = st->iter;
  v.max_iter = st->max_iter;
  v.t_start = st->t_start;
  v.tol_mode = st->tol_mode;
  v.done = st->done;
  return v;
}

// The eight sums that close an iteration -- sum r, sum r^2, sum p phi~,
// sum s, sum s^2, sum q psi~, <C, X> and sum [t]_+^2 -- from the aux
// workgroups' published partials `bp` (slot-major [kSlots][nb]): each lane
// adds a fixed subset in a fixed order, then a DPP reduction; every lane of
// the wave gets the totals.  A column workgroup fills only the column and
// tile slots and a row workgroup the row and tile slots, and the sum skips
// the others.  AGENT: the sums were published by workgroups of the same
// launch (device-scope loads after the acquire fence); otherwise by an
// earlier launch, whose end made them visible to plain (cached) loads.
template <bool AGENT>
__device__ __forceinline__ void iter_sums(const double* bp, int nb, int col_wgs, double (&w)[8]) {
  constexpr int B = 4;  // workgroups per lane in flight
  const int lane = threadIdx.x & (kWave - 1);
  constexpr int slot[8] = {kSR, kSR2, kSPphi, kSS, kSS2, kSQpsi, kST0, kST1};
#pragma unroll
  for (int s = 0; s < 8; ++s) w[s] = 0.0;
  for (int k0 = 0; k0 < nb; k0 += B * kWave) {
    double v[B][8];
#pragma unroll
    for (int u = 0; u < B; ++u) {
#pragma unroll
      for (int s = 0; s < 8; ++s) v[u][s] = 0.0;
      if (k0 + u * kWave >= nb) continue;  // wave-uniform: no load in this block
      const int k = k0 + u * kWave + lane;
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        bool use = k < nb;
        if (s < 3) use = use && k >= col_wgs;
        else if (s < 6) use = use && k < col_wgs;
        const double* ptr = bp + (int64_t)slot[s] * nb + k;
        if (use) v[u][s] = AGENT ? load_agent(ptr) : *ptr;
      }
    }
#pragma unroll
    for (int u = 0; u < B; ++u)
#pragma unroll
      for (int s = 0; s < 8; ++s) w[s] += v[u][s];
  }
  wave_sum_n(w);
}

// The scalar steps closing iteration k = sv.iter + 1 (Algorithm 1 steps
// 5-8, scalar part, and the stopping criteria of Section 3) from the sums w
// of iter_sums and the state sv entering it: beta = f^T r / (m+n), the common
// scalar part 2 beta - alpha of the new shifts, alpha <- alpha - beta, the
// objectives, residuals and the test.  `nc`: the iteration read no C (the
// C-free step of the skip-C schedule), so it has no <C,X> and no dual
// residual: it records NaN for them and can only stop at max_iter.
struct ScalarStep {
  double cphi, cpsi, alpha, pobj, dobj, rp, rd, gap, test;
  int64_t k;
  int done, status;
};

__device__ __forceinline__ ScalarStep scalar_step(const StateIn& sv, const double (&w)[8],
                                                  int64_t m, int64_t n, bool nc) {
  ScalarStep f;
  const double mn = (double)(m + n);
  const double rho = sv.rho;
  const double beta = w[0] / mn;
  const double cc = 2.0 * beta - sv.alpha;
  f.cphi = cc / (double)n;
  f.cpsi = cc / (double)m;
  f.alpha = sv.alpha - beta;
  const double nan = __builtin_nan("");
  f.pobj = nc ? nan : w[6];
  f.dobj = (w[2] + f.cphi * sv.sum_p + w[5] + f.cpsi * sv.sum_q) / rho;
  f.gap = fabs(f.pobj - f.dobj);
  f.rp = sqrt(w[1] + w[4]);
  f.rd = nc ? nan : sqrt(w[7]) / rho;
  const double ep = f.rp / fmax(sv.norm_pq, 1e-300);
  const double ed = f.rd / fmax(sv.norm_c, 1e-300);
  const double eg = f.gap / fmax(fmax(fabs(f.pobj), fabs(f.dobj)), 1e-300);
  f.test = sv.tol_mode ? fmax(f.rp, fmax(f.rd, f.gap)) : fmax(ep, fmax(ed, eg));
  f.k = sv.iter + 1;
  f.done = 0;
  f.status = 0;
  if ((!nc && !finite_d(f.test)) || !finite_d(f.alpha) || !finite_d(cc) || !finite_d(f.rp)) {
    f.done = 1;
    f.status = -3;
  } else if (!nc && f.test <= sv.tol) {
    f.done = 1;
  } else if (f.k >= sv.max_iter) {
    f.done = 1;
    f.status = 1;
  }
  return f;
}

// Write the state after iteration f.k into `dst` (a copy of `src`, the
// record entering it, with the iteration fields replaced) and its trace
// record.  One thread.
__device__ __forceinline__ void commit_step(DevState* dst, const DevState* src,
                                            const ScalarStep& f, const SweepArgs& a,
                                            uint64_t t_start) {
  const uint64_t now = wall_clock64();
  if (dst != src) *dst = *src;
  dst->alpha = f.alpha;
  dst->cphi = f.cphi;
  dst->cpsi = f.cpsi;
  dst->iter = f.k;
  dst->t_last = now;
  dst->pobj = f.pobj;
  dst->dobj = f.dobj;
  dst->rp = f.rp;
  dst->rd = f.rd;
  dst->gap = f.gap;
  dst->test = f.test;
  const int64_t slot = f.k - 1 < a.trace_cap ? f.k - 1 : (f.k - 1) % a.trace_cap;
  double* tr = a.trace + slot * kTraceWidth;
  tr[0] = f.pobj;
  tr[1] = f.dobj;
  tr[2] = f.rp;
  tr[3] = f.rd;
  tr[4] = f.gap;
  tr[5] = f.test;
  tr[6] = (double)(now - t_start) / a.wall_rate;
  tr[7] = (double)f.k;
  if (f.done) {
    dst->done = 1;
    dst->status = f.status;
    dst->stop_iter = f.k;
    dst->t_stop = now;
  }
}

// Run by one wave (all lanes active) once every aux workgroup's sums are in
// `bp`: the last aux workgroup, or a one-wave finishing launch.  Fixed-order
// sum of the workgroups' scalar partials, then, in lane 0, the scalar steps
// of the iteration (from the record `src`, committed to `dst`), of the
// initialisation or of the final evaluation (into `dst`).
template <int MODE>
__device__ void finish_global(const SweepArgs& a, const StateIn& sv, int nb, int col_wgs,
                              const DevState* src, const double* bp, DevState* dst) {
  const int lane = threadIdx.x;
  if (is_iter(MODE)) {
    double w[8];
    iter_sums<true>(bp, nb, col_wgs, w);
    if (lane != 0) return;
    const ScalarStep f = scalar_step(sv, w, a.g.m, a.g.n, MODE == kIterB);
    commit_step(dst, src, f, a, sv.t_start);
    return;
  }
  constexpr int B = 4;  // blockpart columns per lane in flight
  double acc[kSlots];
#pragma unroll
  for (int s = 0; s < kSlots; ++s) acc[s] = 0.0;
  for (int k0 = 0; k0 < nb; k0 += B * kWave) {
    double v[B][kSlots];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int k = k0 + u * kWave + lane;
#pragma unroll
      for (int s = 0; s < kSlots; ++s)
        v[u][s] = k < nb ? load_agent(bp + (int64_t)s * nb + k) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < B; ++u)
#pragma unroll
      for (int s = 0; s < kSlots; ++s) acc[s] += v[u][s];
  }
  wave_sum_n(acc);
  if (lane != 0) return;

  DevState* st = dst;
  const int64_t m = a.g.m, n = a.g.n;
  const double mn = (double)(m + n);
  const double rho = sv.rho;
  const uint64_t now = wall_clock64();
  if (is_final(MODE)) {
    const double pobj = acc[kST0];
    const double dobj = (acc[kSPphi] + acc[kSQpsi]) / rho;
    st->f_pobj = pobj;
    st->f_dobj = dobj;
    st->f_rp = sqrt(acc[kSR2] + acc[kSS2]);
    st->f_rd = sqrt(acc[kST1]) / rho;
    st->f_gap = fabs(pobj - dobj);
    st->f_eps_p = st->f_rp / fmax(sv.norm_pq, 1e-300);
    st->f_eps_d = st->f_rd / fmax(sv.norm_c, 1e-300);
    st->f_eps_g = st->f_gap / fmax(fmax(fabs(pobj), fabs(dobj)), 1e-300);
  } else {
    st->alpha = acc[kSR] / mn;
    st->sum_p = acc[kSP];
    st->sum_q = acc[kSQ];
    st->norm_pq = sqrt(acc[kSPQ2]);
    st->norm_c = sqrt(acc[kST0]);
    st->init_bad = acc[kST1] + acc[kSNonfin];
    st->init_neg = acc[kSNeg];
    st->cphi = 0.0;
    st->cpsi = 0.0;
    st->iter = 0;
    st->done = 0;
    st->status = 0;
    st->stop_iter = 0;
    st->t_last = now;
  }
}

// Loads of a strided sequence (base[r * stride], r0 <= r < r1) added into
// `s` in ascending r, with the loads issued in masked batches of U so that a
// short sequence costs one memory latency.
template <int U, typename V, int CW>
__device__ __forceinline__ void sum_strided(const V* base, int64_t stride, int r0, int r1,
                                            double (&s)[CW]) {
  for (int rb = r0; rb < r1; rb += U) {
    V v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int r = rb + u;
      v[u] = r < r1 ? __builtin_nontemporal_load(base + (int64_t)r * stride) : V{};
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int e = 0; e < CW; ++e) s[e] += (double)v[u][e];
  }
}

// ---------------------------------------------------------------------------
// The O(m+n) kernel.  Workgroups [0, col_wgs) own kAuxCols columns each: the
// column partials are read as 16-byte chunks with the row groups split over
// G thread groups, then combined in LDS in a fixed order.  The remaining
// workgroups own kAuxRows rows each, with the column strips' row partials
// split over the four waves.  All loads are issued up front, in masked
// batches, ahead of the stop flag's test.  Every scalar contribution (the
// per-column or per-row terms and a fixed slice of the tile scalars) lives in
// wave 0, which sums them with DPP, publishes them and takes part in the
// last-workgroup election; the other waves leave after the loads.  Wave 0 of
// the last workgroup does the scalar steps.
// ---------------------------------------------------------------------------
template <typename T, int MODE, bool WIDE = false, bool SPLIT = false>
__device__ __forceinline__ void aux_body(const SweepArgs& a, const int b, const int nb) {
  using P = typename std::conditional<WIDE, double, typename PartialOf<T, MODE>::type>::type;
  constexpr int CW = 16 / sizeof(P);      // columns per 16-byte chunk
  constexpr int NCH = kAuxCols / CW;      // chunks per workgroup
  constexpr int G = kBlock / NCH;         // row-group groups
  using V = typename VecOf<P, CW>::type;
  static_assert(G * kAuxCols >= kWaves * kAuxRows, "LDS buffer holds the row partials");
  static_assert(kAuxCols <= kWave && kAuxRows == kWave, "wave 0 finishes the entries");

  const StateIn sv = load_state(a.st);
  __shared__ double red2[G * kAuxCols];

  const int64_t m = a.g.m, n = a.g.n;
  const int col_wgs = (int)((n + kAuxCols - 1) / kAuxCols);
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const bool is_col = b < col_wgs;

  // Stage 1: loads.  `idx` is the column (column workgroups, threads below
  // kAuxCols) or row (row workgroups, wave 0) this thread finishes, else -1;
  // `w0`, `w1` its marginal entry and its accumulator (or phi / psi, or the
  // warm start).
  int64_t idx = -1;
  double w0 = 0.0, w1 = 0.0;
  if (is_col) {
    const int64_t j0 = (int64_t)b * kAuxCols;
    const int ch = threadIdx.x % NCH, grp = threadIdx.x / NCH;
    const int n_rg = a.g.n_rg;
    const int r0 = (int)((int64_t)n_rg * grp / G), r1 = (int)((int64_t)n_rg * (grp + 1) / G);
    const P* cp = static_cast<const P*>(a.colpart) + j0 + ch * CW;
    double s[CW];
#pragma unroll
    for (int e = 0; e < CW; ++e) s[e] = 0.0;
    sum_strided<8>(reinterpret_cast<const V*>(cp), a.g.ldcp / CW, r0, r1, s);
#pragma unroll
    for (int e = 0; e < CW; ++e) red2[grp * kAuxCols + ch * CW + e] = s[e];
    const int64_t j = j0 + threadIdx.x;
    if (threadIdx.x < kAuxCols && j < n) {
      idx = j;
      w0 = (double)static_cast<const T*>(a.q)[j];
      if (is_iter(MODE)) w1 = a.b[j];
      else if (is_final(MODE)) w1 = a.psi64[j];
      else w1 = a.nu0 ? a.nu0[j] : 0.0;
    }
  } else {
    const int64_t i = (int64_t)(b - col_wgs) * kAuxRows + lane;
    double u[1] = {0.0};
    if (i < m) {
      const int n_ct = a.g.n_ct;
      const int c0 = n_ct * wave / kWaves, c1 = n_ct * (wave + 1) / kWaves;
      typedef P P1 __attribute__((ext_vector_type(1)));
      sum_strided<8>(reinterpret_cast<const P1*>(static_cast<const P*>(a.rowpart) + i), m, c0, c1,
                     u);
      if (wave == 0) {
        idx = i;
        w0 = (double)static_cast<const T*>(a.p)[i];
        if (is_iter(MODE)) w1 = a.a[i];
        else if (is_final(MODE)) w1 = a.phi64[i];
        else w1 = a.mu0 ? a.mu0[i] : 0.0;
      }
    }
    red2[wave * kAuxRows + lane] = u[0];
  }
  double acc[kSlots];
#pragma unroll
  for (int s = 0; s < kSlots; ++s) acc[s] = 0.0;
  if (wave == 0) {
    // A fixed slice of the sweep's tile scalars, 4 tiles per lane in flight.
    const int64_t nt = (int64_t)a.g.n_ct * a.g.n_rg;
    const int64_t t0 = nt * b / nb, t1 = nt * (b + 1) / nb;
    for (int64_t tb = t0; tb < t1; tb += 4 * kWave) {
      double v0[4], v1[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t t = tb + u * kWave + lane;
        v0[u] = t < t1 ? a.tiles[t * kTileSlots + kTs0] : 0.0;
        v1[u] = t < t1 ? a.tiles[t * kTileSlots + kTs1] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        acc[kST0] += v0[u];
        acc[kST1] += v1[u];
      }
    }
  }
  __syncthreads();
  if (wave != 0 || (is_iter(MODE) && sv.done)) return;

  // Stage 2 (wave 0): the per-entry steps, written once for both kinds of
  // workgroup: `tot` is the entry's full sum (u_i or v_j), `len` the length
  // of the other side (n for rows, m for columns).  The three pointers are
  // picked as values (made wave-uniform first), so that no field of the
  // arguments is ever addressed through a runtime choice.
  const double rho = sv.rho;
  double* const accv = pick(is_col, a.b, a.a);      // a_i or b_j
  double* const d64 = pick(is_col, a.psi64, a.phi64);
  T* const dT = static_cast<T*>(pick(is_col, a.psiT, a.phiT));
  double* const dout = pick(is_col, a.nu_out, a.mu_out);
  const double len = is_col ? (double)m : (double)n;
  const double shift = is_col ? sv.cpsi : sv.cphi;
  const double sum0 = is_col ? sv.sum_phi0 : sv.sum_psi0;
  // e0, e1, e2: the entry's (residual or a_0 / b_0, its square, marginal x dual)
  double e0 = 0.0, e1 = 0.0, e2 = 0.0, emarg = 0.0, esq = 0.0, eneg = 0.0, ebad = 0.0;
  if (idx >= 0) {
    double tot;
    if (is_col) {
      tot = red2[threadIdx.x];
#pragma unroll
      for (int g = 1; g < G; ++g) tot += red2[g * kAuxCols + threadIdx.x];
    } else {
      tot = red2[lane];
#pragma unroll
      for (int w = 1; w < kWaves; ++w) tot += red2[w * kAuxRows + lane];
    }
    const double marg = w0;
    const double res = tot - marg;
    if (is_iter(MODE)) {
      const double d = (w1 - 2.0 * res) / len;
      accv[idx] = w1 - res;
      d64[idx] = d;
      dT[idx] = (T)d;
      e0 = res;
      e1 = res * res;
      e2 = marg * d;
    } else if (is_final(MODE)) {
      const double d = w1 + shift;
      e1 = res * res;
      e2 = marg * d;
      if (dout) dout[idx] = d / rho;
    } else {
      const double d0 = rho * w1;
      const double acc0 = res + len * d0 + sum0;
      accv[idx] = acc0;
      d64[idx] = d0;
      dT[idx] = (T)d0;
      e0 = acc0;
      emarg = marg;
      esq = marg * marg;
      eneg = marg < 0.0 ? 1.0 : 0.0;
      ebad = (!finite_d(marg) || !finite_d(d0)) ? 1.0 : 0.0;
    }
  }

  // Publish this workgroup's sums (slot-major), then count it in; the
  // release fence orders the stores before the count and the acquire fence
  // of the last workgroup orders its loads after it.  Column workgroups fill
  // the column slots, row workgroups the row slots; in the iteration no
  // other slot is read.
  double* const bp = a.blockpart + b;
  const int64_t sb = is_col ? kSS : kSR;  // first of the side's three slots
  unsigned prev = 0;
  if (is_iter(MODE)) {
    double w[5] = {e0, e1, e2, acc[kST0], acc[kST1]};
    wave_sum_n(w);
    if (lane == 0) {
      store_agent(bp + (sb + 0) * nb, w[0]);
      store_agent(bp + (sb + 1) * nb, w[1]);
      store_agent(bp + (sb + 2) * nb, w[2]);
      store_agent(bp + (int64_t)kST0 * nb, w[3]);
      store_agent(bp + (int64_t)kST1 * nb, w[4]);
    }
  } else {
    // Initialisation / final evaluation: all 13 slots, zeros included.
    double w[10] = {e0, e1, e2, emarg, esq, eneg, ebad, acc[kST0], acc[kST1], 0.0};
    wave_sum_n(w);
    const double r0 = is_col ? 0.0 : w[0], r1 = is_col ? 0.0 : w[1], r2 = is_col ? 0.0 : w[2];
    const double c0 = is_col ? w[0] : 0.0, c1 = is_col ? w[1] : 0.0, c2 = is_col ? w[2] : 0.0;
    const double sp = is_col ? 0.0 : w[3], sq = is_col ? w[3] : 0.0;
    if (lane == 0) {
      store_agent(bp + (int64_t)kSR * nb, r0);
      store_agent(bp + (int64_t)kSR2 * nb, r1);
      store_agent(bp + (int64_t)kSPphi * nb, r2);
      store_agent(bp + (int64_t)kSS * nb, c0);
      store_agent(bp + (int64_t)kSS2 * nb, c1);
      store_agent(bp + (int64_t)kSQpsi * nb, c2);
      store_agent(bp + (int64_t)kST0 * nb, w[7]);
      store_agent(bp + (int64_t)kST1 * nb, w[8]);
      store_agent(bp + (int64_t)kSP * nb, sp);
      store_agent(bp + (int64_t)kSQ * nb, sq);
      store_agent(bp + (int64_t)kSPQ2 * nb, w[4]);
      store_agent(bp + (int64_t)kSNeg * nb, w[5]);
      store_agent(bp + (int64_t)kSNonfin * nb, w[6]);
    }
  }
  // Split form: the scalar steps run in a separate one-workgroup launch, and
  // the kernel boundary publishes the sums (no fence per workgroup).
  if constexpr (SPLIT) return;
  if (lane == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    prev = __hip_atomic_fetch_add(&a.st->counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  prev = __builtin_amdgcn_readfirstlane(prev);
  if (prev != (unsigned)(nb - 1)) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  finish_global<MODE>(a, sv, nb, col_wgs, a.st, a.blockpart, a.st);
  if (lane == 0)
    __hip_atomic_store(&a.st->counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T, int MODE, bool WIDE = false, bool SPLIT = false>
__global__ __launch_bounds__(kBlock) void aux_kernel(SweepArgs a) {
  aux_body<T, MODE, WIDE, SPLIT>(a, blockIdx.x, gridDim.x);
}

// The scalar steps after a publish-only aux launch: one wave.  They read the
// record and sums of the aux launch (a.st, a.blockpart), or in the pending
// form (a.st_prev, a.bp_prev), and commit into a.st.
template <int MODE>
__device__ __forceinline__ void finish_body(const SweepArgs& a) {
  const DevState* src = a.st_prev ? a.st_prev : a.st;
  const double* bp = a.st_prev ? a.bp_prev : a.blockpart;
  const StateIn sv = load_state(src);
  if (is_iter(MODE) && sv.done) {
    if (src != a.st && threadIdx.x == 0) *a.st = *src;  // carry the stopped state forward
    return;
  }
  const int nb = (int)aux_workgroups(a.g.m, a.g.n);
  const int col_wgs = (int)((a.g.n + kAuxCols - 1) / kAuxCols);
  finish_global<MODE>(a, sv, nb, col_wgs, src, bp, a.st);
}

template <int MODE>
__global__ __launch_bounds__(kWave) void finish_kernel(SweepArgs a) {
  finish_body<MODE>(a);
}

// Batched form: one wave per problem (finished problems return at once).
template <int MODE>
__global__ __launch_bounds__(kWave) void finish_batch_kernel(const SweepArgs* __restrict__ args) {
  const SweepArgs a = args[blockIdx.x];
  finish_body<MODE>(a);
}

// ---------------------------------------------------------------------------
// Small problems: the whole iteration in one workgroup of kSmallBlock
// threads, `iters` iterations per launch.  Below a few hundred kilobytes per
// iteration the two-launch iteration is bound by the fixed cost of its
// launches and of its dependent memory round trips, not by bandwidth; here
// the plan and the cost stay in registers for the whole launch and three
// workgroup barriers per iteration are the only synchronisation.  Same
// steps, state and stopping test as sweep + aux:
//  - wave w holds rows w, w + 16, ... (RT of them), lane l the columns
//    l, l + 64, ... (NCOL of them); step 4 on these entries, with the row
//    and column partials combined in LDS in a fixed order;
//  - thread i finishes row i and thread j column j (steps 5-8);
//  - wave 0 combines the eight scalar sums in a fixed order and takes the
//    scalar step (the shifts of step 3, alpha, the stopping test), and
//    broadcasts it through LDS.
// The workgroup runs on one compute unit, so the cost of an iteration is
// its instruction count: work that only one wave needs runs in one wave,
// and a row's sum goes through LDS (each lane's partial, added up by the
// row's thread) instead of a DPP reduction per row.  Each lane's partial
// sums (of at most 32 entries) are in the problem's type, as in the sweep;
// everything after them is float64.
// ---------------------------------------------------------------------------

// Sum over each row of 16 lanes (fixed order); every lane of the row gets it.
__device__ __forceinline__ double row16_sum(double v) {
  v += dpp<0xB1>(v);   // pairs
  v += dpp<0x4E>(v);   // quads
  v += dpp<0x141>(v);  // half-row mirror: 8
  v += dpp<0x140>(v);  // row mirror: 16
  return v;
}

__device__ __forceinline__ double read_lane(double v, int l) {
  const unsigned long long bits = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = __builtin_amdgcn_readlane((int)(unsigned)(bits & 0xffffffffull), l);
  const unsigned hi = __builtin_amdgcn_readlane((int)(unsigned)(bits >> 32), l);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

template <typename T, int NCOL>
__global__ __launch_bounds__(kSmallBlock) void small_kernel(SweepArgs a, int64_t iters) {
  constexpr int NW = kSmallWaves;
  constexpr int RT = small_slots(std::is_same<T, float>::value ? 0 : 1) / NCOL;
  constexpr int NC = kWave * NCOL;  // columns covered
  __shared__ T rowsh[NW * RT];
  __shared__ T colsh[NC];
  __shared__ T rowp[NW * RT][kWave];  // each lane's partial of each row
  __shared__ double colp[NW][NC];
  __shared__ double red[NW][8];
  // Per-row and per-column vectors of steps 5-8 (a, phi~, p and b, psi~, q),
  // each entry used only by its own thread; kept here to free registers.
  __shared__ double rv[3][NW * RT];
  __shared__ double cv[3][NC];
  __shared__ double rec[6];  // the latest iteration's record, from thread 0
  __shared__ double bc[4];   // the scalar step's results, from thread 0

  DevState* st = a.st;
  const StateIn sv = load_state(st);
  if (sv.done) return;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const int m = (int)a.g.m, n = (int)a.g.n;
  const int64_t ldc = a.g.ldc, ldx = a.g.ldx;
  const T* __restrict__ C = static_cast<const T*>(a.C);
  T* __restrict__ X = static_cast<T*>(a.X);
  const double rho = sv.rho;
  const T rhoT = (T)rho;
  const bool own_r = tid < m, own_c = tid < n;
  // rows held by this wave: wave + NW t for t < nrows
  const int nrows = m > wave ? (m - wave + NW - 1) / NW : 0;
  bool jv[NCOL];
#pragma unroll
  for (int c = 0; c < NCOL; ++c) jv[c] = lane + kWave * c < n;

  T xr[RT][NCOL], cr[RT][NCOL];
#pragma unroll
  for (int t = 0; t < RT; ++t) {
    const int64_t i = wave + NW * t;
#pragma unroll
    for (int c = 0; c < NCOL; ++c) {
      const int j = lane + kWave * c;
      const bool v = t < nrows && jv[c];
      xr[t][c] = v ? X[i * ldx + j] : (T)0;
      cr[t][c] = v ? C[i * ldc + j] : (T)0;
    }
  }

  if (own_r) {
    rv[0][tid] = a.a[tid];
    rv[1][tid] = a.phi64[tid];
    rv[2][tid] = (double)static_cast<const T*>(a.p)[tid];
    rowsh[tid] = static_cast<const T*>(a.phiT)[tid];
  }
  if (own_c) {
    cv[0][tid] = a.b[tid];
    cv[1][tid] = a.psi64[tid];
    cv[2][tid] = (double)static_cast<const T*>(a.q)[tid];
  }
  if (tid < NC) colsh[tid] = own_c ? static_cast<const T*>(a.psiT)[tid] : (T)0;
  double alpha = sv.alpha, cphi = sv.cphi, cpsi = sv.cpsi;
  int64_t k = sv.iter;
  int done = 0, status = 0;
  __syncthreads();

  for (int64_t it = 0; it < iters; ++it) {
    // Step 4 on the held entries, with the row sums, the column partials
    // and the stopping-test partials <C,X> and |[.]_+|^2.
    const T shift = (T)(cphi + cpsi);
    T colv[NCOL];
#pragma unroll
    for (int c = 0; c < NCOL; ++c) colv[c] = colsh[lane + kWave * c];
    T cacc[NCOL];
#pragma unroll
    for (int c = 0; c < NCOL; ++c) cacc[c] = (T)0;
    T s0 = (T)0, s1 = (T)0;
    // The cost is loop-invariant; without this the compiler hoists rho c and
    // its float64 widening out of the loop, which needs three times the
    // registers and spills.
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int c = 0; c < NCOL; ++c) asm volatile("" : "+v"(cr[t][c]));
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      if (t < nrows) {
        const T rowv = rowsh[wave + NW * t] + shift;
        T rs = (T)0;
#pragma unroll
        for (int c = 0; c < NCOL; ++c) {
          if (jv[c]) {
            const T tt = rowv + colv[c] - mul_rounded<T>(rhoT, cr[t][c]);
            const T tp = tt > (T)0 ? tt : (T)0;
            s1 += tp * tp;
            const T y = xr[t][c] + tt;
            const T xn = y > (T)0 ? y : (T)0;
            xr[t][c] = xn;
            rs += xn;
            cacc[c] += xn;
            s0 += cr[t][c] * xn;
          }
        }
        rowp[wave + NW * t][lane] = rs;
      }
    }
#pragma unroll
    for (int c = 0; c < NCOL; ++c) colp[wave][lane + kWave * c] = (double)cacc[c];
    __syncthreads();

    // Steps 5-8 per row and column, and the eight scalar sums.  Waves with
    // no row or column owner only reduce their sweep partials.
    if (wave * kWave < (m > n ? m : n)) {
      double e[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, (double)s0, (double)s1};
      if (own_r) {
        // the row's 64 lane partials, in four interleaved chains; thread i
        // starts at lane i mod 64 so that the threads of a wave read
        // different banks
        double u4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
        for (int u0 = 0; u0 < kWave; u0 += 8) {
          T v8[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) v8[u] = rowp[tid][(u0 + u + tid) & (kWave - 1)];
#pragma unroll
          for (int u = 0; u < 8; ++u) u4[u & 3] += (double)v8[u];
        }
        const double usum = (u4[0] + u4[1]) + (u4[2] + u4[3]);
        const double ai = rv[0][tid], pi = rv[2][tid];
        const double r = usum - pi;
        const double ph = (ai - 2.0 * r) / (double)n;
        rv[0][tid] = ai - r;
        rv[1][tid] = ph;
        rowsh[tid] = (T)ph;
        e[0] = r;
        e[1] = r * r;
        e[2] = pi * ph;
      }
      if (own_c) {
        double v = colp[0][tid];
#pragma unroll
        for (int w = 1; w < NW; ++w) v += colp[w][tid];
        const double bj = cv[0][tid], qj = cv[2][tid];
        const double s = v - qj;
        const double ps = (bj - 2.0 * s) / (double)m;
        cv[0][tid] = bj - s;
        cv[1][tid] = ps;
        colsh[tid] = (T)ps;
        e[3] = s;
        e[4] = s * s;
        e[5] = qj * ps;
      }
      wave_sum_n(e);
      if (lane == 0)
#pragma unroll
        for (int q = 0; q < 8; ++q) red[wave][q] = e[q];
    } else {
      double e[2] = {(double)s0, (double)s1};
      wave_sum_n(e);
      if (lane == 0) {
#pragma unroll
        for (int q = 0; q < 6; ++q) red[wave][q] = 0.0;
        red[wave][6] = e[0];
        red[wave][7] = e[1];
      }
    }
    __syncthreads();

    // The scalar step in wave 0: lane l adds red[l % 16][l / 16] and
    // red[l % 16][4 + l / 16] over its row of 16 lanes (a fixed order).
    if (wave == 0) {
      const double v0 = row16_sum(red[lane & 15][lane >> 4]);
      const double v1 = row16_sum(red[lane & 15][4 + (lane >> 4)]);
      double acc[8];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        acc[q] = read_lane(v0, 16 * q);
        acc[4 + q] = read_lane(v1, 16 * q);
      }
      const double beta = acc[0] / (double)(m + n);
      const double cc = 2.0 * beta - alpha;
      const double nphi = cc / (double)n, npsi = cc / (double)m;
      const double pobj = acc[6];
      const double dobj = (acc[2] + nphi * sv.sum_p + acc[5] + npsi * sv.sum_q) / rho;
      const double gap = fabs(pobj - dobj);
      const double rp = sqrt(acc[1] + acc[4]);
      const double rd = sqrt(acc[7]) / rho;
      const double ep = rp / fmax(sv.norm_pq, 1e-300);
      const double ed = rd / fmax(sv.norm_c, 1e-300);
      const double eg = gap / fmax(fmax(fabs(pobj), fabs(dobj)), 1e-300);
      const double test = sv.tol_mode ? fmax(rp, fmax(rd, gap)) : fmax(ep, fmax(ed, eg));
      const double alpha_next = alpha - beta;
      const int64_t kn = k + 1;
      int dn = 0;
      if (!finite_d(test) || !finite_d(alpha_next) || !finite_d(cc) || !finite_d(rp)) {
        dn = 1;
        status = -3;
      } else if (test <= sv.tol) {
        dn = 1;
        status = 0;
      } else if (kn >= sv.max_iter) {
        dn = 1;
        status = 1;
      }
      if (lane == 0) {
        const uint64_t now = wall_clock64();
        const int64_t slot = kn - 1 < a.trace_cap ? kn - 1 : (kn - 1) % a.trace_cap;
        double* tr = a.trace + slot * kTraceWidth;
        tr[0] = pobj;
        tr[1] = dobj;
        tr[2] = rp;
        tr[3] = rd;
        tr[4] = gap;
        tr[5] = test;
        tr[6] = (double)(now - sv.t_start) / a.wall_rate;
        tr[7] = (double)kn;
        rec[0] = pobj;
        rec[1] = dobj;
        rec[2] = rp;
        rec[3] = rd;
        rec[4] = gap;
        rec[5] = test;
        bc[0] = nphi;
        bc[1] = npsi;
        bc[2] = alpha_next;
        bc[3] = (double)dn;
      }
    }
    __syncthreads();
    cphi = bc[0];
    cpsi = bc[1];
    alpha = bc[2];
    done = bc[3] != 0.0;
    ++k;
    if (done) break;
  }

  // A fresh base for the stores, so that the load addresses are not kept
  // live (in registers or scratch) through the iteration.
  T* Xw = X;
  int64_t ldw = ldx;
  int lw = lane, ww = wave;
  asm volatile("" : "+s"(Xw), "+s"(ldw), "+v"(lw), "+v"(ww));
#pragma unroll
  for (int t = 0; t < RT; ++t) {
    const int64_t i = ww + NW * t;
#pragma unroll
    for (int c = 0; c < NCOL; ++c)
      if (t < nrows && jv[c]) Xw[i * ldw + lw + kWave * c] = xr[t][c];
  }
  if (own_r) {
    a.a[tid] = rv[0][tid];
    a.phi64[tid] = rv[1][tid];
    static_cast<T*>(a.phiT)[tid] = (T)rv[1][tid];
  }
  if (own_c) {
    a.b[tid] = cv[0][tid];
    a.psi64[tid] = cv[1][tid];
    static_cast<T*>(a.psiT)[tid] = (T)cv[1][tid];
  }
  if (tid == 0) {
    const uint64_t now = wall_clock64();
    st->alpha = alpha;
    st->cphi = cphi;
    st->cpsi = cpsi;
    st->iter = k;
    st->t_last = now;
    if (k > sv.iter) {
      st->pobj = rec[0];
      st->dobj = rec[1];
      st->rp = rec[2];
      st->rd = rec[3];
      st->gap = rec[4];
      st->test = rec[5];
    }
    if (done) {
      st->done = 1;
      st->status = status;
      st->stop_iter = k;
      st->t_stop = now;
    }
  }
}

// Batched form: work item = (problem, aux workgroup of that problem).
template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void aux_batch_kernel(const SweepArgs* __restrict__ args,
                                                           const uint2* __restrict__ work) {
  const uint2 w = work[blockIdx.x];
  // A private copy of the problem's arguments: read through the pointer,
  // every field would be reloaded after each store the kernel makes.
  const SweepArgs a = args[__builtin_amdgcn_readfirstlane(w.x)];
  aux_body<T, MODE, false, true>(a, (int)w.y, (int)aux_workgroups(a.g.m, a.g.n));
}

// The batched iteration's aux work items, one per wave, four per workgroup
// (the batch's items are small: a few row groups deep, so a whole workgroup
// per item spent most of its life on fixed costs).  Per item the same
// quantities as aux_body<T, kIter, false, true> with these orders: column
// items split the row groups over G1 lane groups (each adds its range in
// order) and add the G1 sums in order; row items add their strips in order;
// every lane then takes the step of its column or row.
template <typename T>
__device__ __forceinline__ void aux_wave_iter(const SweepArgs& a, const int b, const int nb,
                                              double* __restrict__ red) {
  using P = typename PartialOf<T, kIter>::type;
  constexpr int CW = 16 / sizeof(P);   // columns per 16-byte chunk
  constexpr int NCH = kAuxCols / CW;   // chunks per item
  constexpr int G1 = kWave / NCH;      // row-group ranges per item (= CW)
  using V = typename VecOf<P, CW>::type;
  static_assert(kAuxCols == kWave && kAuxRows == kWave, "one entry per lane");

  const StateIn sv = load_state(a.st);
  const int64_t m = a.g.m, n = a.g.n;
  const int col_wgs = (int)((n + kAuxCols - 1) / kAuxCols);
  const int lane = threadIdx.x & (kWave - 1);
  const bool is_col = b < col_wgs;

  int64_t idx = -1;
  double w0 = 0.0, w1 = 0.0, tot = 0.0;
  if (is_col) {
    const int64_t j0 = (int64_t)b * kAuxCols;
    const int ch = lane % NCH, grp = lane / NCH;
    const int n_rg = a.g.n_rg;
    const int r0 = (int)((int64_t)n_rg * grp / G1), r1 = (int)((int64_t)n_rg * (grp + 1) / G1);
    const P* cp = static_cast<const P*>(a.colpart) + j0 + ch * CW;
    double sv4[CW];
#pragma unroll
    for (int e = 0; e < CW; ++e) sv4[e] = 0.0;
    sum_strided<8>(reinterpret_cast<const V*>(cp), a.g.ldcp / CW, r0, r1, sv4);
#pragma unroll
    for (int e = 0; e < CW; ++e) red[grp * kAuxCols + ch * CW + e] = sv4[e];
    const int64_t j = j0 + lane;
    if (j < n) {
      idx = j;
      w0 = (double)static_cast<const T*>(a.q)[j];
      w1 = a.b[j];
    }
  } else {
    const int64_t i = (int64_t)(b - col_wgs) * kAuxRows + lane;
    if (i < m) {
      typedef P P1 __attribute__((ext_vector_type(1)));
      double u[1] = {0.0};
      sum_strided<8>(reinterpret_cast<const P1*>(static_cast<const P*>(a.rowpart) + i), m, 0,
                     a.g.n_ct, u);
      tot = u[0];
      idx = i;
      w0 = (double)static_cast<const T*>(a.p)[i];
      w1 = a.a[i];
    }
  }
  // A fixed slice of the sweep's tile scalars.
  double st0 = 0.0, st1 = 0.0;
  {
    const int64_t nt = (int64_t)a.g.n_ct * a.g.n_rg;
    const int64_t t0 = nt * b / nb, t1 = nt * (b + 1) / nb;
    for (int64_t tb = t0; tb < t1; tb += 4 * kWave) {
      double v0[4], v1[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t t = tb + u * kWave + lane;
        v0[u] = t < t1 ? a.tiles[t * kTileSlots + kTs0] : 0.0;
        v1[u] = t < t1 ? a.tiles[t * kTileSlots + kTs1] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        st0 += v0[u];
        st1 += v1[u];
      }
    }
  }
  if (sv.done) return;
  // The column sums cross lanes of this wave through LDS.
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (is_col && idx >= 0) {
    tot = red[lane];
#pragma unroll
    for (int g = 1; g < G1; ++g) tot += red[g * kAuxCols + lane];
  }
  double* const accv = pick(is_col, a.b, a.a);      // a_i or b_j
  double* const d64 = pick(is_col, a.psi64, a.phi64);
  T* const dT = static_cast<T*>(pick(is_col, a.psiT, a.phiT));
  const double len = is_col ? (double)m : (double)n;
  double e0 = 0.0, e1 = 0.0, e2 = 0.0;
  if (idx >= 0) {
    const double res = tot - w0;
    const double d = (w1 - 2.0 * res) / len;
    accv[idx] = w1 - res;
    d64[idx] = d;
    dT[idx] = (T)d;
    e0 = res;
    e1 = res * res;
    e2 = w0 * d;
  }
  double w[5] = {e0, e1, e2, st0, st1};
  wave_sum_n(w);
  if (lane == 0) {
    double* const bp = a.blockpart + b;
    const int64_t sb = is_col ? kSS : kSR;
    store_agent(bp + (sb + 0) * nb, w[0]);
    store_agent(bp + (sb + 1) * nb, w[1]);
    store_agent(bp + (sb + 2) * nb, w[2]);
    store_agent(bp + (int64_t)kST0 * nb, w[3]);
    store_agent(bp + (int64_t)kST1 * nb, w[4]);
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void aux_batch_iter_kernel(const SweepArgs* __restrict__ args,
                                                                const uint2* __restrict__ work,
                                                                int64_t n_aux) {
  constexpr int CW = 16 / sizeof(typename PartialOf<T, kIter>::type);
  __shared__ double red[kWaves][CW * kAuxCols];  // per wave: CW row-group ranges x 64 columns
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int64_t item = (int64_t)blockIdx.x * kWaves + wave;
  if (item >= n_aux) return;
  const uint2 w = work[item];
  const SweepArgs a = args[__builtin_amdgcn_readfirstlane(w.x)];  // private copy, as above
  aux_wave_iter<T>(a, (int)__builtin_amdgcn_readfirstlane(w.y), (int)aux_workgroups(a.g.m, a.g.n),
                   red[wave]);
}

// Per-lane accumulator of the sweep.  Plain: a running sum in the partial
// type.  Compensated (float32 iteration with DROT_FLAG_COMPENSATED): a
// Neumaier (improved Kahan-Babuska) pair of floats, so that a lane's sum over
// its entries carries an error of about one rounding whatever its length; the
// pair is handed on as s + c in float64, and every later combination
// (across lanes, waves, tiles) is a float64 sum.
template <typename P, bool KC>
struct LaneAcc {
  P v = 0;
  template <typename X>
  __device__ __forceinline__ void add(X x) { v += (P)x; }
  __device__ __forceinline__ P get() const { return v; }
};

template <>
struct LaneAcc<double, true> {
  float s = 0.f, c = 0.f;
  __device__ __forceinline__ void add(float x) {
    const float t = s + x;
    c += __builtin_fabsf(s) >= __builtin_fabsf(x) ? (s - t) + x : (x - t) + s;
    s = t;
  }
  __device__ __forceinline__ double get() const { return (double)s + (double)c; }
};

// ---------------------------------------------------------------------------
// The sweep.  A workgroup owns one column strip of W = 64 * VEC * CH columns
// and the row blocks g, g + G, g + 2G, ... of `rows` rows each (G = n_rg row
// groups): the workgroups running at any moment stream one contiguous band
// of row blocks (short blocks keep DRAM pages open), while column partials
// are kept per group, so there are G rows of them instead of one per block.
// Within a block the four waves take contiguous slices of rows; each lane
// owns CH chunks of VEC consecutive columns and keeps the loads of U rows in
// flight.  Consecutive workgroups take consecutive strips of the same group.
// ---------------------------------------------------------------------------
template <typename T, int MODE, int VEC, int CH, int U, bool NT, int CM, int D, bool RAGGED,
          bool KC = false>
__device__ __forceinline__ void sweep_body(const SweepArgs& a, const int ct, const int rg) {
  static_assert(!KC || (std::is_same<T, float>::value && MODE == kIter),
                "compensated sums: float32 plain iteration only");
  using P = typename std::conditional<KC, double, typename PartialOf<T, MODE>::type>::type;
  using L = LaneAcc<P, KC>;
  using A = typename std::conditional<is_final(MODE), double, T>::type;
  constexpr int CPL = VEC * CH;
  constexpr int W = kWave * CPL;
  constexpr bool kReadC = MODE != kIterB && CM != kCostCoords;
  static_assert(CM == kCostDense || std::is_same<T, float>::value, "cost kind needs float32");
  constexpr bool kReadX = MODE != kInitPQ;
  constexpr bool kWriteX = MODE != kInitX && MODE != kFinal;

  // The state entering this iteration.  Pending form (a.st_prev set): every
  // wave closes the previous iteration itself from its record and its aux
  // sums (the same fixed-order arithmetic everywhere, so every workgroup
  // takes the same shift and the same stop decision), and workgroup 0
  // commits the result to a.st, which no other workgroup reads here.
  const int64_t m = a.g.m, n = a.g.n;
  const DevState* st = is_iter(MODE) && a.st_prev ? a.st_prev : a.st;
  double shift_d = 0.0;
  if (is_iter(MODE)) {
    if (a.st_prev) {
      // Wave 0 closes the previous iteration and hands the shift and the
      // stop decision to the other waves through LDS.
      __shared__ double closing[2];
      if (threadIdx.x < kWave) {
        // The record's loads first, so that they are in flight with the sums'.
        const StateIn pv = load_state(a.st_prev);
        double w[8];
        iter_sums<false>(a.bp_prev, (int)aux_workgroups(m, n),
                         (int)((n + kAuxCols - 1) / kAuxCols), w);
        double sh = 0.0, stop = 1.0;
        if (pv.done) {
          if (blockIdx.x == 0 && threadIdx.x == 0) *a.st = *a.st_prev;
        } else {
          const ScalarStep f = scalar_step(pv, w, m, n, a.prev_b != 0);
          if (blockIdx.x == 0 && threadIdx.x == 0) commit_step(a.st, a.st_prev, f, a, pv.t_start);
          sh = f.cphi + f.cpsi;
          stop = f.done ? 1.0 : 0.0;
        }
        if (threadIdx.x == 0) {
          closing[0] = sh;
          closing[1] = stop;
        }
      }
      __syncthreads();
      if (closing[1] != 0.0) return;
      shift_d = closing[0];
    } else {
      if (st->done) return;
      shift_d = st->cphi + st->cpsi;
    }
  } else if (is_final(MODE)) {
    shift_d = st->cphi + st->cpsi;
  }

  const int lane = threadIdx.x & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int64_t col0 = (int64_t)ct * W;
  const int rpw = (a.g.rows + kWaves - 1) / kWaves;

  const T* __restrict__ C = static_cast<const T*>(a.C);
  const uint16_t* __restrict__ Cb = static_cast<const uint16_t*>(a.C);
  T* __restrict__ X = static_cast<T*>(a.X);

  // Column layout of this lane: chunk c covers [jc[c], jc[c] + VEC), of which
  // nv[c] columns lie inside the matrix.  A chunk that straddles column n is
  // loaded whole (the leading dimensions are multiples of VEC, so the load
  // stays inside the row) but only its valid elements count and are stored.
  int64_t jc[CH];
  int nv[CH];
  bool ok[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    jc[c] = col0 + (int64_t)c * kWave * VEC + (int64_t)lane * VEC;
    const int64_t left = n - jc[c];
    if constexpr (RAGGED) nv[c] = left <= 0 ? 0 : (left >= VEC ? VEC : (int)left);
    else nv[c] = left > 0 ? VEC : 0;  // n is a multiple of VEC
    ok[c] = nv[c] > 0;
  }

  // Column shift of this lane's columns (or q_j for X_0 = p q^T).
  A colv[CH][VEC];
#pragma unroll
  for (int c = 0; c < CH; ++c)
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      A v = 0;
      if (e < nv[c]) {
        const int64_t j = jc[c] + e;
        if (is_iter(MODE)) v = static_cast<const T*>(a.psiT)[j];
        if (is_final(MODE)) v = a.psi64[j];
        if (MODE == kInitPQ) v = static_cast<const T*>(a.q)[j];
      }
      colv[c][e] = v;
    }

  // Coordinates of this lane's target points (coordinates cost only).
  constexpr int DD = CM == kCostCoords ? D : 1;
  float xtl[CH][VEC][DD];
  float cscale = 0.f;
  if constexpr (CM == kCostCoords) {
    cscale = (float)st->cscale;
#pragma unroll
    for (int c = 0; c < CH; ++c)
#pragma unroll
      for (int e = 0; e < VEC; ++e)
#pragma unroll
        for (int d = 0; d < D; ++d) xtl[c][e][d] = e < nv[c] ? a.xt[(jc[c] + e) * D + d] : 0.f;
  }

  A shift = 0, rho = 0;
  T rhoT = 0;
  if (is_iter(MODE) || is_final(MODE)) {
    shift = (A)shift_d;
    rho = (A)st->rho;
    rhoT = (T)st->rho;
  }

  L colacc[CH][VEC];
  L s0, s1;  // tile scalars (cost & dual, or |C|^2 & bad count)

  P* __restrict__ rowpart = static_cast<P*>(a.rowpart);

  for (int64_t rb = rg; rb < a.g.n_rb; rb += a.g.n_rg) {
  const int64_t row0 = rb * a.g.rows;
  const int64_t rowE = row0 + a.g.rows < m ? row0 + a.g.rows : m;
  const int64_t rw0 = row0 + (int64_t)wave * rpw;
  const int64_t rw1 = rw0 + rpw < rowE ? rw0 + rpw : rowE;
  for (int64_t i0 = rw0; i0 < rw1; i0 += U) {
    T xv[U][CH][VEC], cv[U][CH][VEC];
    float xsr[U][DD];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + u;
      if (i < rw1) {
        if constexpr (CM == kCostCoords)
#pragma unroll
          for (int d = 0; d < D; ++d) xsr[u][d] = a.xs[i * D + d];
#pragma unroll
        for (int c = 0; c < CH; ++c) {
          if (ok[c]) {
            if constexpr (kReadC && CM == kCostDense)
              load_chunk<T, VEC, NT>(C + i * a.g.ldc + jc[c], cv[u][c]);
            if constexpr (kReadC && CM == kCostBF16)
              load_bf16<VEC, NT>(Cb + i * a.g.ldc + jc[c], cv[u][c]);
            if (kReadX) load_chunk<T, VEC, NT>(X + i * a.g.ldx + jc[c], xv[u][c]);
          }
        }
      }
    }
    // c_ij as the storage type sees it.
    auto cost = [&](int u, int c, int e) -> T {
      if constexpr (CM == kCostCoords) {
        float s = 0.f;
#pragma unroll
        for (int d = 0; d < D; ++d) {
          const float df = xsr[u][d] - xtl[c][e][d];
          s += df * df;
        }
        return (T)(s * cscale);
      } else {
        return cv[u][c][e];
      }
    };
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + u;
      if (i < rw1) {
        A rowv = 0;
        if (is_iter(MODE)) rowv = static_cast<const T*>(a.phiT)[i] + shift;
        if (is_final(MODE)) rowv = a.phi64[i] + (double)shift;
        if (MODE == kInitPQ) rowv = static_cast<const T*>(a.p)[i];
        L rsum;
#pragma unroll
        for (int c = 0; c < CH; ++c) {
          if (ok[c]) {
            T outv[VEC];
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
              A x = 0;
              if (RAGGED && e >= nv[c]) {
                // beyond column n (padding): contributes nothing, never stored
                outv[e] = (T)0;
              } else if constexpr (MODE == kIterB) {
                // X_{k+2} = [W + phi_i + psi_j]_+ with W = X_{k+1} - rho C.
                const A y = (A)xv[u][c][e] + (rowv + colv[c][e]);
                x = y > (A)0 ? y : (A)0;
                outv[e] = (T)x;
              } else if constexpr (is_iter(MODE) || is_final(MODE)) {
                const A cij = (A)cost(u, c, e);
                const A pc = is_final(MODE) ? rho * cij : mul_rounded<A>(rho, cij);
                const A t = rowv + colv[c][e] - pc;
                const A tp = t > (A)0 ? t : (A)0;
                s1.add(tp * tp);
                if constexpr (MODE == kFinalW) {
                  // Restore X from W in the stored type, with the product the
                  // C-reading iteration subtracted.
                  const T pcT = mul_rounded<T>(rhoT, cv[u][c][e]);
                  const T xr = xv[u][c][e] + pcT;
                  outv[e] = xr;
                  x = (A)xr;
                } else if constexpr (MODE == kFinal) {
                  x = (A)xv[u][c][e];
                } else {
                  const A y = (A)xv[u][c][e] + t;
                  x = y > (A)0 ? y : (A)0;
                  outv[e] = MODE == kIterA ? (T)(x - pc) : (T)x;
                }
                s0.add(cij * x);
              } else {
                const A cij = (A)cost(u, c, e);
                if (MODE == kInitPQ) x = rowv * colv[c][e];
                else x = (A)xv[u][c][e];
                s0.add((double)cij * (double)cij);
                const bool bad = !finite_d((double)cij) || !finite_d((double)x) ||
                                 (MODE == kInitX && x < (A)0);
                s1.add(bad ? (P)1 : (P)0);
                outv[e] = (T)x;
              }
              rsum.add(x);
              colacc[c][e].add(x);
            }
            if (kWriteX) {
              if (!RAGGED || nv[c] == VEC) {
                store_chunk<T, VEC, NT>(X + i * a.g.ldx + jc[c], outv);
              } else {
#pragma unroll
                for (int e = 0; e < VEC; ++e)
                  if (e < nv[c]) X[i * a.g.ldx + jc[c] + e] = outv[e];
              }
            }
          }
        }
        const P tot = wave_sum(rsum.get());
        if (lane == 0) rowpart[(int64_t)ct * m + i] = tot;
      }
    }
  }
  }

  // ---- tile partials: combine the four waves in LDS, fixed order -----------
  __shared__ P sm[kWaves * W];
  __shared__ double ssc[2][kWaves];
#pragma unroll
  for (int c = 0; c < CH; ++c)
#pragma unroll
    for (int e = 0; e < VEC; ++e)
      sm[wave * W + c * kWave * VEC + lane * VEC + e] = colacc[c][e].get();
  const P w0 = wave_sum(s0.get());
  const P w1 = wave_sum(s1.get());
  if (lane == 0) {
    ssc[0][wave] = (double)w0;
    ssc[1][wave] = (double)w1;
  }
  __syncthreads();
  P* __restrict__ colpart = static_cast<P*>(a.colpart);
  for (int k = threadIdx.x; k < W; k += kBlock) {
    const int64_t j = col0 + k;
    if (j < n) {
      P v = sm[k];
#pragma unroll
      for (int w = 1; w < kWaves; ++w) v += sm[w * W + k];
      colpart[(int64_t)rg * a.g.ldcp + j] = v;
    }
  }
  if (threadIdx.x == 0) {
    double v0 = ssc[0][0], v1 = ssc[1][0];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) {
      v0 += ssc[0][w];
      v1 += ssc[1][w];
    }
    double* t = a.tiles + ((int64_t)rg * a.g.n_ct + ct) * kTileSlots;
    t[kTs0] = v0;
    t[kTs1] = v1;
  }
}

template <typename T, int MODE, int VEC, int CH, int U, bool NT, int CM, int D, bool RAGGED,
          bool KC>
__global__ __launch_bounds__(kBlock) void sweep_kernel(SweepArgs a) {
  sweep_body<T, MODE, VEC, CH, U, NT, CM, D, RAGGED, KC>(a, blockIdx.x % a.g.n_ct,
                                                          blockIdx.x / a.g.n_ct);
}

// Batched form: work item = (problem, workgroup of that problem's sweep).
template <typename T, int MODE, int VEC, int CH, bool NT, bool RAGGED>
__global__ __launch_bounds__(kBlock) void sweep_batch_kernel(const SweepArgs* __restrict__ args,
                                                             const uint2* __restrict__ work) {
  const uint2 w = work[blockIdx.x];
  const SweepArgs a = args[__builtin_amdgcn_readfirstlane(w.x)];  // private copy, as above
  sweep_body<T, MODE, VEC, CH, 4, NT, kCostDense, 1, RAGGED>(a, (int)(w.y % a.g.n_ct),
                                                              (int)(w.y / a.g.n_ct));
}

// Warm-start sums sum(phi_0) = rho sum(mu0), sum(psi_0) = rho sum(nu0), the
// start timestamp, and zeroed completion counters.  One workgroup.
__device__ __forceinline__ void prep_body(const SweepArgs& a) {
  __shared__ double red[kSlots][kWaves];
  double acc[kSlots];
#pragma unroll
  for (int s = 0; s < kSlots; ++s) acc[s] = 0.0;
  if (a.mu0)
    for (int64_t i = threadIdx.x; i < a.g.m; i += kBlock) acc[0] += a.mu0[i];
  if (a.nu0)
    for (int64_t j = threadIdx.x; j < a.g.n; j += kBlock) acc[1] += a.nu0[j];
  block_sum_slots(acc, red);
  if (threadIdx.x == 0) {
    DevState* st = a.st;
    st->sum_phi0 = st->rho * acc[0];
    st->sum_psi0 = st->rho * acc[1];
    if (a.cost_kind == kCostCoords && !(st->cscale > 0.0)) {
      const float mx = __uint_as_float(st->maxc_bits);
      st->cscale = mx > 0.f ? 1.0 / (double)mx : 1.0;
    }
    st->t_start = wall_clock64();
    st->t_stop = st->t_start;
    st->t_last = st->t_start;
    st->counter = 0;
  }
}

__global__ __launch_bounds__(kBlock) void prep_kernel(SweepArgs a) { prep_body(a); }

__global__ __launch_bounds__(kBlock) void prep_batch_kernel(const SweepArgs* __restrict__ args) {
  const SweepArgs a = args[blockIdx.x];
  prep_body(a);
}

// Stream of a sweep launch, with optional events that hipExtLaunchKernel
// stamps with the dispatch's own start and end times.
struct Launch {
  hipStream_t s;
  hipEvent_t e0, e1;
};

template <typename T, int MODE, int VEC, int CH, int U, bool NT, int CM = kCostDense, int D = 1,
          bool RAGGED = false, bool KC = false>
hipError_t sweep_go(const SweepArgs& a, const Launch& s) {
  const dim3 grid((unsigned)((int64_t)a.g.n_ct * a.g.n_rg));
  if (s.e0 || s.e1)
    hipExtLaunchKernelGGL((sweep_kernel<T, MODE, VEC, CH, U, NT, CM, D, RAGGED, KC>), grid,
                          dim3(kBlock), 0, s.s, s.e0, s.e1, 0, a);
  else
    hipLaunchKernelGGL((sweep_kernel<T, MODE, VEC, CH, U, NT, CM, D, RAGGED, KC>), grid,
                       dim3(kBlock), 0, s.s, a);
  return hipGetLastError();
}

// The compensated float32 iteration: 16-byte path with 1 or 2 chunks, 4 rows
// in flight, cached or streaming; the scalar path with 4 chunks (which the
// host also uses for ragged widths).
template <int CM, int D>
hipError_t sweep_comp(const TileCfg& t, const SweepArgs& a, const Launch& s) {
  if (t.ragged || t.unroll != 4) return hipErrorInvalidValue;
  if (t.vec == 1) {
    if (t.chunks != 4) return hipErrorInvalidValue;
    return sweep_go<float, kIter, 1, 4, 4, false, CM, D, false, true>(a, s);
  }
  if (t.vec != 4) return hipErrorInvalidValue;
  switch ((t.chunks == 2 ? 1 : 0) | (t.stream ? 2 : 0)) {
    case 0: return sweep_go<float, kIter, 4, 1, 4, false, CM, D, false, true>(a, s);
    case 1: return sweep_go<float, kIter, 4, 2, 4, false, CM, D, false, true>(a, s);
    case 2: return sweep_go<float, kIter, 4, 1, 4, true, CM, D, false, true>(a, s);
    case 3: return sweep_go<float, kIter, 4, 2, 4, true, CM, D, false, true>(a, s);
  }
  return hipErrorInvalidValue;
}

// 16-byte path with n not a multiple of the vector width (masked last chunk):
// 1 or 2 chunks, 4 rows in flight, cached or streaming.
template <typename T, int MODE, int CM, int D>
hipError_t sweep_ragged(const TileCfg& t, const SweepArgs& a, const Launch& s) {
  constexpr int V = 16 / sizeof(T);
  if (t.vec != V || t.unroll != 4) return hipErrorInvalidValue;
  switch ((t.chunks == 2 ? 1 : 0) | (t.stream ? 2 : 0)) {
    case 0: return sweep_go<T, MODE, V, 1, 4, false, CM, D, true>(a, s);
    case 1: return sweep_go<T, MODE, V, 2, 4, false, CM, D, true>(a, s);
    case 2: return sweep_go<T, MODE, V, 1, 4, true, CM, D, true>(a, s);
    case 3: return sweep_go<T, MODE, V, 2, 4, true, CM, D, true>(a, s);
  }
  return hipErrorInvalidValue;
}

// The iteration instantiates every tile variant; initialisation and the final
// evaluation run once per solve and use the plain 4-row variant.
template <typename T, int MODE>
hipError_t sweep_dense(const TileCfg& t, const SweepArgs& a, const Launch& s) {
  constexpr int V = 16 / sizeof(T);
  if (t.ragged) return sweep_ragged<T, MODE, kCostDense, 1>(t, a, s);
  if (t.vec == 1) {
    if (t.chunks == 1) return sweep_go<T, MODE, 1, 1, 4, false>(a, s);
    if (t.chunks == 4) return sweep_go<T, MODE, 1, 4, 4, false>(a, s);
    return hipErrorInvalidValue;
  }
  if (t.vec != V) return hipErrorInvalidValue;
  if constexpr (is_iter(MODE)) {
    const int key = (t.chunks == 2 ? 1 : 0) | (t.unroll == 8 ? 2 : 0) | (t.stream ? 4 : 0);
    switch (key) {
      case 0: return sweep_go<T, MODE, V, 1, 4, false>(a, s);
      case 1: return sweep_go<T, MODE, V, 2, 4, false>(a, s);
      case 2: return sweep_go<T, MODE, V, 1, 8, false>(a, s);
      case 3: return sweep_go<T, MODE, V, 2, 8, false>(a, s);
      case 4: return sweep_go<T, MODE, V, 1, 4, true>(a, s);
      case 5: return sweep_go<T, MODE, V, 2, 4, true>(a, s);
      case 6: return sweep_go<T, MODE, V, 1, 8, true>(a, s);
      case 7: return sweep_go<T, MODE, V, 2, 8, true>(a, s);
    }
    return hipErrorInvalidValue;
  } else {
    if (t.chunks == 1) return sweep_go<T, MODE, V, 1, 4, false>(a, s);
    if (t.chunks == 2) return sweep_go<T, MODE, V, 2, 4, false>(a, s);
    return hipErrorInvalidValue;
  }
}

// Non-dense cost sources (float32 only): 1 or 2 chunks, 4 rows in flight,
// cached or streaming; the scalar path uses 4 chunks, cached.
template <int MODE, int CM, int D>
hipError_t sweep_cost(const TileCfg& t, const SweepArgs& a, const Launch& s) {
  if (t.ragged) return sweep_ragged<float, MODE, CM, D>(t, a, s);
  if (t.vec == 1) {
    if (t.chunks == 4) return sweep_go<float, MODE, 1, 4, 4, false, CM, D>(a, s);
    return hipErrorInvalidValue;
  }
  if (t.vec != 4 || t.unroll != 4) return hipErrorInvalidValue;
  const int key = (t.chunks == 2 ? 1 : 0) | (t.stream ? 2 : 0);
  switch (key) {
    case 0: return sweep_go<float, MODE, 4, 1, 4, false, CM, D>(a, s);
    case 1: return sweep_go<float, MODE, 4, 2, 4, false, CM, D>(a, s);
    case 2: return sweep_go<float, MODE, 4, 1, 4, true, CM, D>(a, s);
    case 3: return sweep_go<float, MODE, 4, 2, 4, true, CM, D>(a, s);
  }
  return hipErrorInvalidValue;
}

template <typename T, int MODE>
hipError_t sweep_mode(const TileCfg& t, const SweepArgs& a, const Launch& s) {
  if (t.comp) {
    if constexpr (std::is_same<T, float>::value && MODE == kIter) {
      switch (a.cost_kind) {
        case kCostDense: return sweep_comp<kCostDense, 1>(t, a, s);
        case kCostBF16: return sweep_comp<kCostBF16, 1>(t, a, s);
        case kCostCoords:
          if (a.dim == 1) return sweep_comp<kCostCoords, 1>(t, a, s);
          if (a.dim == 2) return sweep_comp<kCostCoords, 2>(t, a, s);
          if (a.dim == 3) return sweep_comp<kCostCoords, 3>(t, a, s);
      }
      return hipErrorInvalidValue;
    }
    // Initialisation and the final evaluation already accumulate in float64.
    if constexpr (MODE == kIter || MODE == kIterA || MODE == kIterB) return hipErrorInvalidValue;
  }
  if (a.cost_kind == kCostDense) return sweep_dense<T, MODE>(t, a, s);
  if constexpr (std::is_same<T, float>::value && !(MODE == kIterA || MODE == kIterB ||
                                                   MODE == kFinalW)) {
    if (a.cost_kind == kCostBF16) return sweep_cost<MODE, kCostBF16, 1>(t, a, s);
    if (a.cost_kind == kCostCoords) {
      switch (a.dim) {
        case 1: return sweep_cost<MODE, kCostCoords, 1>(t, a, s);
        case 2: return sweep_cost<MODE, kCostCoords, 2>(t, a, s);
        case 3: return sweep_cost<MODE, kCostCoords, 3>(t, a, s);
      }
    }
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t sweep_type(int mode, const TileCfg& t, const SweepArgs& a, const Launch& s) {
  switch (mode) {
    case kIter: return sweep_mode<T, kIter>(t, a, s);
    case kInitPQ: return sweep_mode<T, kInitPQ>(t, a, s);
    case kInitX: return sweep_mode<T, kInitX>(t, a, s);
    case kFinal: return sweep_mode<T, kFinal>(t, a, s);
    case kIterA: return sweep_mode<T, kIterA>(t, a, s);
    case kIterB: return sweep_mode<T, kIterB>(t, a, s);
    case kFinalW: return sweep_mode<T, kFinalW>(t, a, s);
  }
  return hipErrorInvalidValue;
}

// max_ij |xs_i - xt_j|^2 for the coordinates cost (scale = 1 / max when the
// caller gives none).  A block covers 256 targets and up to 256 sources; the
// maximum of nonnegative floats is taken on their bit patterns, which order
// the same way, so the result does not depend on the order of the atomics.
template <int D>
__global__ __launch_bounds__(kBlock) void maxc_kernel(SweepArgs a) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.y * kBlock;
  const int64_t i1 = i0 + kBlock < a.g.m ? i0 + kBlock : a.g.m;
  float mx = 0.f;
  if (j < a.g.n) {
    float yt[D];
#pragma unroll
    for (int d = 0; d < D; ++d) yt[d] = a.xt[j * D + d];
    for (int64_t i = i0; i < i1; ++i) {
      float s = 0.f;
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const float df = a.xs[i * D + d] - yt[d];
        s += df * df;
      }
      mx = s > mx ? s : mx;
    }
  }
  for (int off = kWave / 2; off > 0; off /= 2) {
    const float o = __shfl_xor(mx, off);
    mx = o > mx ? o : mx;
  }
  if ((threadIdx.x & (kWave - 1)) == 0) atomicMax(&a.st->maxc_bits, __float_as_uint(mx));
}

// One aux launch in the form chosen by the workgroup count: with many
// workgroups the last-arriving election costs one L2 write-back per workgroup
// (its release fence), so above kAuxSplitMin workgroups the aux kernel only
// publishes its sums and a one-wave kernel does the scalar steps.
template <typename T, int MODE, bool WIDE>
hipError_t aux_go(const SweepArgs& a, hipStream_t s, bool publish) {
  const int64_t nb = aux_workgroups(a.g.m, a.g.n);
  const dim3 grid((unsigned)nb);
  if (publish) {
    hipLaunchKernelGGL((aux_kernel<T, MODE, WIDE, true>), grid, dim3(kBlock), 0, s, a);
  } else if (nb >= kAuxSplitMin) {
    hipLaunchKernelGGL((aux_kernel<T, MODE, WIDE, true>), grid, dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL((finish_kernel<MODE>), dim3(1), dim3(kWave), 0, s, a);
  } else {
    hipLaunchKernelGGL((aux_kernel<T, MODE, WIDE, false>), grid, dim3(kBlock), 0, s, a);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t aux_type(int mode, bool wide, const SweepArgs& a, hipStream_t s, bool publish) {
  if (publish && !is_iter(mode)) return hipErrorInvalidValue;
  if (wide && std::is_same<T, float>::value) {
    // Float64 partials of the compensated float32 iteration.
    if (mode != kIter) return hipErrorInvalidValue;
    return aux_go<T, kIter, true>(a, s, publish);
  }
  switch (mode) {
    case kIter:
    case kIterA: return aux_go<T, kIter, false>(a, s, publish);
    case kIterB: return aux_go<T, kIterB, false>(a, s, publish);
    case kInitPQ:
    case kInitX: return aux_go<T, kInitPQ, false>(a, s, false);
    case kFinal:
    case kFinalW: return aux_go<T, kFinal, false>(a, s, false);
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_aux(int dtype, int mode, const SweepArgs& a, hipStream_t s, bool wide,
                      bool publish) {
  return dtype == 0 ? aux_type<float>(mode, wide, a, s, publish)
                    : aux_type<double>(mode, wide, a, s, publish);
}

hipError_t launch_finish(int mode, const SweepArgs& a, hipStream_t s) {
  if (mode == kIter || mode == kIterA)
    hipLaunchKernelGGL((finish_kernel<kIter>), dim3(1), dim3(kWave), 0, s, a);
  else if (mode == kIterB)
    hipLaunchKernelGGL((finish_kernel<kIterB>), dim3(1), dim3(kWave), 0, s, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_sweep(int dtype, int mode, const TileCfg& t, const SweepArgs& a,
                        hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  const Launch L{s, e0, e1};
  return dtype == 0 ? sweep_type<float>(mode, t, a, L) : sweep_type<double>(mode, t, a, L);
}

namespace {

template <typename T, int MODE>
hipError_t sweep_batch_mode(const TileCfg& t, const SweepArgs* args, const uint2* work,
                            int64_t nwork, hipStream_t s) {
  constexpr int V = 16 / sizeof(T);
  const dim3 grid((unsigned)nwork), block(kBlock);
  if (t.vec == 1 && t.chunks == 4) {
    hipLaunchKernelGGL((sweep_batch_kernel<T, MODE, 1, 4, false, false>), grid, block, 0, s, args, work);
    return hipGetLastError();
  }
  if (t.vec != V || t.unroll != 4) return hipErrorInvalidValue;
  switch ((t.chunks == 2 ? 1 : 0) | (t.stream ? 2 : 0)) {
    case 0: hipLaunchKernelGGL((sweep_batch_kernel<T, MODE, V, 1, false, true>), grid, block, 0, s, args, work); break;
    case 1: hipLaunchKernelGGL((sweep_batch_kernel<T, MODE, V, 2, false, true>), grid, block, 0, s, args, work); break;
    case 2: hipLaunchKernelGGL((sweep_batch_kernel<T, MODE, V, 1, true, true>), grid, block, 0, s, args, work); break;
    case 3: hipLaunchKernelGGL((sweep_batch_kernel<T, MODE, V, 2, true, true>), grid, block, 0, s, args, work); break;
  }
  return hipGetLastError();
}

// Batched aux: every workgroup publishes its sums, then one wave per problem
// does the scalar steps (a per-workgroup release fence would cost one L2
// write-back per workgroup of every problem).
template <typename T, int MODE>
void batch_aux(const SweepArgs* args, const uint2* aux_work, int64_t n_aux, int n_prob,
               hipStream_t s) {
  if constexpr (MODE == kIter)
    hipLaunchKernelGGL((aux_batch_iter_kernel<T>), dim3((unsigned)((n_aux + kWaves - 1) / kWaves)),
                       dim3(kBlock), 0, s, args, aux_work, n_aux);
  else
    hipLaunchKernelGGL((aux_batch_kernel<T, MODE>), dim3((unsigned)n_aux), dim3(kBlock), 0, s, args,
                       aux_work);
  hipLaunchKernelGGL((finish_batch_kernel<MODE>), dim3((unsigned)n_prob), dim3(kWave), 0, s, args);
}

template <typename T>
hipError_t batch_type(int mode, const TileCfg& t, const SweepArgs* args, const uint2* sweep_work,
                      int64_t n_sweep, const uint2* aux_work, int64_t n_aux, int n_prob,
                      hipStream_t s) {
  hipError_t e = hipSuccess;
  switch (mode) {
    case kIter:
      e = sweep_batch_mode<T, kIter>(t, args, sweep_work, n_sweep, s);
      if (e == hipSuccess) batch_aux<T, kIter>(args, aux_work, n_aux, n_prob, s);
      break;
    case kInitPQ:
    case kInitX:
      e = mode == kInitPQ ? sweep_batch_mode<T, kInitPQ>(t, args, sweep_work, n_sweep, s)
                          : sweep_batch_mode<T, kInitX>(t, args, sweep_work, n_sweep, s);
      if (e == hipSuccess) batch_aux<T, kInitPQ>(args, aux_work, n_aux, n_prob, s);
      break;
    case kFinal:
      e = sweep_batch_mode<T, kFinal>(t, args, sweep_work, n_sweep, s);
      if (e == hipSuccess) batch_aux<T, kFinal>(args, aux_work, n_aux, n_prob, s);
      break;
    default: return hipErrorInvalidValue;
  }
  return e != hipSuccess ? e : hipGetLastError();
}

}  // namespace

hipError_t launch_batch_step(int dtype, int mode, const TileCfg& t, const SweepArgs* args,
                             const uint2* sweep_work, int64_t n_sweep, const uint2* aux_work,
                             int64_t n_aux, int n_prob, hipStream_t s) {
  if (n_sweep <= 0 || n_aux <= 0) return hipSuccess;
  return dtype == 0
             ? batch_type<float>(mode, t, args, sweep_work, n_sweep, aux_work, n_aux, n_prob, s)
             : batch_type<double>(mode, t, args, sweep_work, n_sweep, aux_work, n_aux, n_prob, s);
}

hipError_t launch_prep_batch(const SweepArgs* args, int count, hipStream_t s) {
  hipLaunchKernelGGL(prep_batch_kernel, dim3((unsigned)count), dim3(kBlock), 0, s, args);
  return hipGetLastError();
}

namespace {
template <typename T>
hipError_t small_type(const SweepArgs& a, int64_t iters, hipStream_t s) {
  const dim3 grid(1), block(kSmallBlock);
  switch (small_cols(a.g.n)) {
    case 1: hipLaunchKernelGGL((small_kernel<T, 1>), grid, block, 0, s, a, iters); break;
    case 2: hipLaunchKernelGGL((small_kernel<T, 2>), grid, block, 0, s, a, iters); break;
    case 4: hipLaunchKernelGGL((small_kernel<T, 4>), grid, block, 0, s, a, iters); break;
    case 8: hipLaunchKernelGGL((small_kernel<T, 8>), grid, block, 0, s, a, iters); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
}  // namespace

hipError_t launch_small(int dtype, const SweepArgs& a, int64_t iters, hipStream_t s) {
  // The kernel's register and LDS arrays are sized for small_fits shapes.
  if (!small_fits(dtype, a.g.m, a.g.n)) return hipErrorInvalidValue;
  return dtype == 0 ? small_type<float>(a, iters, s) : small_type<double>(a, iters, s);
}

hipError_t launch_maxc(const SweepArgs& a, hipStream_t s) {
  const dim3 grid((unsigned)((a.g.n + kBlock - 1) / kBlock), (unsigned)((a.g.m + kBlock - 1) / kBlock));
  switch (a.dim) {
    case 1: hipLaunchKernelGGL(maxc_kernel<1>, grid, dim3(kBlock), 0, s, a); break;
    case 2: hipLaunchKernelGGL(maxc_kernel<2>, grid, dim3(kBlock), 0, s, a); break;
    case 3: hipLaunchKernelGGL(maxc_kernel<3>, grid, dim3(kBlock), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_prep(const SweepArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(prep_kernel, dim3(1), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

}  // namespace drot

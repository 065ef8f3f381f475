// A small multilayer perceptron trained with hand-written gfx950 kernels:
// the learned warm start of DROT.  It maps the marginals (p, q) of an OT
// problem to initial dual variables (mu, nu); DROT then starts from the shifts
// phi_0 = rho mu, psi_0 = rho nu (a warm start is valid because DR converges
// from any starting point, Lemma 1).
//
// Network: in -> hidden (ReLU) -> hidden (ReLU) -> out, mean-squared-error
// loss.  Weights are kept in float32 (Adam master copy) and bfloat16 (the
// copy the matrix cores read); activations and gradients enter the GEMMs in
// bfloat16 and every GEMM accumulates in float32 on the MFMA units
// (v_mfma_f32_32x32x8 bf16).  All reductions run in a fixed order.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/drot.h"

int drot_internal_fail(int code, const char* msg);

namespace {

int mfail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  return drot_internal_fail(code, buf);
}

#define MHIP(expr)                                                                   \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess)                                                            \
      return mfail(DROT_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));     \
  } while (0)

typedef uint16_t bf16;
typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));

__host__ __device__ inline bf16 to_bf16(float f) {
  // round to nearest even (finite inputs)
  uint32_t u;
  memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (bf16)(u >> 16);
}

// ---------------------------------------------------------------------------
// C[M x N] = op(A)[M x K] * op(B)[K x N] (+ beta * C), bfloat16 inputs,
// float32 accumulation on the matrix cores (v_mfma_f32_32x32x8 bf16).  A is
// stored row-major as M x K (TA = 0) or K x M (TA = 1); B as K x N (TB = 0)
// or N x K (TB = 1).  A workgroup of four waves computes a 64 x 64 tile, each
// wave a 32 x 32 block; K advances 32 at a time.  Every thread brings one
// 16-byte piece (8 bfloat16 along the stored contiguous dimension) of each
// operand tile into LDS, where both tiles are kept K-contiguous (As[m][k],
// Bs[n][k]) so that each lane reads its 4-element fragments as 8 bytes.
// Epilogues: EPI 0 stores the product (adding beta * C); EPI 1 adds the bias
// of the column, applies ReLU when `relu`, and stores the float32 result and
// its bfloat16 copy (a layer's forward step); EPI 2 keeps the product where
// `gate` > 0 and zeroes it elsewhere, storing float32 and bfloat16 (the
// backward step through a ReLU).
// EPI 3 (split K): workgroup z of the grid's third dimension multiplies the
// slice [z ks, (z + 1) ks) of K and stores its raw product at C + z M ldc;
// splitk_reduce adds the slices in order and applies the epilogue.
// Requires M % 64 == N % 64 == ks % 32 == 0, leading dimensions multiples of
// 8 and 16-byte aligned operands (checked on the host).
// ---------------------------------------------------------------------------
typedef short v8s __attribute__((ext_vector_type(8)));

template <int TA, int TB, int EPI>
__global__ __launch_bounds__(256) void gemm_bf16(const bf16* __restrict__ A, const bf16* __restrict__ B,
                                                 float* __restrict__ C, int M, int N, int K, int lda,
                                                 int ldb, int ldc, float beta,
                                                 const float* __restrict__ bias,
                                                 const float* __restrict__ gate,
                                                 bf16* __restrict__ Cb, int relu, int ks) {
  constexpr int LDK = 32 + 8;  // K-contiguous rows, 80 bytes: 16-byte stores stay aligned
  __shared__ __align__(16) bf16 As[64][LDK];
  __shared__ __align__(16) bf16 Bs[64][LDK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int wr = wave >> 1, wc = wave & 1;
  v16f acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.f;
  const int kb = blockIdx.z * ks, ke = kb + ks;
  for (int k0 = kb; k0 < ke; k0 += 32) {
    if (TA == 0) {  // row m0 + r of A, k0 + c .. + 7
      const int r = tid >> 2, c = (tid & 3) * 8;
      *reinterpret_cast<v8s*>(&As[r][c]) =
          *reinterpret_cast<const v8s*>(A + (size_t)(m0 + r) * lda + k0 + c);
    } else {        // row k0 + kr of the K x M storage, columns m0 + mc .. + 7
      const int kr = tid >> 3, mc = (tid & 7) * 8;
      const v8s v = *reinterpret_cast<const v8s*>(A + (size_t)(k0 + kr) * lda + m0 + mc);
#pragma unroll
      for (int e = 0; e < 8; ++e) As[mc + e][kr] = (bf16)v[e];
    }
    if (TB == 1) {  // row n0 + r of the N x K storage, k0 + c .. + 7
      const int r = tid >> 2, c = (tid & 3) * 8;
      *reinterpret_cast<v8s*>(&Bs[r][c]) =
          *reinterpret_cast<const v8s*>(B + (size_t)(n0 + r) * ldb + k0 + c);
    } else {        // row k0 + kr of the K x N storage, columns n0 + nc .. + 7
      const int kr = tid >> 3, nc = (tid & 7) * 8;
      const v8s v = *reinterpret_cast<const v8s*>(B + (size_t)(k0 + kr) * ldb + n0 + nc);
#pragma unroll
      for (int e = 0; e < 8; ++e) Bs[nc + e][kr] = (bf16)v[e];
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 32; kk += 8) {
      const v4s a = *reinterpret_cast<const v4s*>(&As[wr * 32 + (lane & 31)][kk + 4 * (lane >> 5)]);
      const v4s b = *reinterpret_cast<const v4s*>(&Bs[wc * 32 + (lane & 31)][kk + 4 * (lane >> 5)]);
      acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  // lane holds column (lane % 32) and rows 8 (r / 4) + 4 (lane / 32) + r % 4
  const int col = n0 + wc * 32 + (lane & 31);
  const float bcol = EPI == 1 ? bias[col] : 0.f;
  if (EPI == 3) C += (size_t)blockIdx.z * M * ldc;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = m0 + wr * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    const size_t o = (size_t)row * ldc + col;
    if (EPI == 3) {
      C[o] = acc[r];
    } else if (EPI == 0) {
      C[o] = acc[r] + (beta != 0.f ? beta * C[o] : 0.f);
    } else {
      float v = acc[r];
      if (EPI == 1) {
        v += bcol;
        if (relu && !(v > 0.f)) v = 0.f;
      } else if (!(gate[o] > 0.f)) {
        v = 0.f;
      }
      C[o] = v;
      Cb[o] = to_bf16(v);
    }
  }
}

// The split-K sum: C = sum over z = 0, 1, ... of P[z] (M x N slices, leading
// dimension N, added in that order), then GEMM epilogue EPI (0, 1 or 2).
template <int EPI>
__global__ __launch_bounds__(256) void splitk_reduce(const float* __restrict__ P, int S, int M,
                                                     int N, float* __restrict__ C, int ldc,
                                                     float beta, const float* __restrict__ bias,
                                                     const float* __restrict__ gate,
                                                     bf16* __restrict__ Cb, int relu) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)M * N) return;
  const int row = (int)(i / N), col = (int)(i % N);
  float v = P[i];
  for (int z = 1; z < S; ++z) v += P[(size_t)z * M * N + i];
  const size_t o = (size_t)row * ldc + col;
  if (EPI == 0) {
    C[o] = v + (beta != 0.f ? beta * C[o] : 0.f);
    return;
  }
  if (EPI == 1) {
    v += bias[col];
    if (relu && !(v > 0.f)) v = 0.f;
  } else if (!(gate[o] > 0.f)) {
    v = 0.f;
  }
  C[o] = v;
  Cb[o] = to_bf16(v);
}

// Mean squared error: dy = 2 (y - t) / count; per-block partial sums of
// (y - t)^2 in float64 (fixed order), summed by the host.
__global__ void mse_grad(const float* __restrict__ y, const float* __restrict__ t,
                         float* __restrict__ dy, bf16* __restrict__ dyb, double* __restrict__ part,
                         int64_t count) {
  __shared__ double red[256];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double s = 0.0;
  if (i < count) {
    const float d = y[i] - t[i];
    const float g = 2.f * d / (float)count;
    dy[i] = g;
    dyb[i] = to_bf16(g);
    s = (double)d * (double)d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Column sums of a rows x cols float32 matrix (bias gradients), fixed order:
// a workgroup owns 64 columns; its kColSlices waves each add the rows
// congruent to the wave index (mod kColSlices), four loads in flight, and
// wave 0 adds the slices' sums in slice order.
constexpr int kColSlices = 16;
__global__ __launch_bounds__(kColSlices * 64) void col_sum(const float* __restrict__ g,
                                                           float* __restrict__ out, int rows,
                                                           int cols) {
  __shared__ float part[kColSlices][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + lane;
  float s = 0.f;
  if (j < cols) {
    int r = w;
    for (; r + 3 * kColSlices < rows; r += 4 * kColSlices) {
      const float v0 = g[(int64_t)r * cols + j];
      const float v1 = g[(int64_t)(r + kColSlices) * cols + j];
      const float v2 = g[(int64_t)(r + 2 * kColSlices) * cols + j];
      const float v3 = g[(int64_t)(r + 3 * kColSlices) * cols + j];
      s += v0;
      s += v1;
      s += v2;
      s += v3;
    }
    for (; r < rows; r += kColSlices) s += g[(int64_t)r * cols + j];
  }
  part[w][lane] = s;
  __syncthreads();
  if (w == 0 && j < cols) {
    float t = 0.f;
#pragma unroll
    for (int k = 0; k < kColSlices; ++k) t += part[k][lane];
    out[j] = t;
  }
}

__global__ void cast_bf16(const float* __restrict__ x, bf16* __restrict__ y, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) y[i] = to_bf16(x[i]);
}

// Adam on the float32 master weights; refreshes the bfloat16 copy.  The
// coefficients b1, 1 - b1, b2, 1 - b2 and the bias corrections c1, c2 come
// from the host rounded once from float64 (1 - b2 formed in float32 from the
// rounded b2 would be 1.3e-5 off).
__global__ void adam(float* __restrict__ w, bf16* __restrict__ wb, const float* __restrict__ g,
                     float* __restrict__ m1, float* __restrict__ m2, int64_t count, float lr,
                     float b1, float ob1, float b2, float ob2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float a = b1 * m1[i] + ob1 * gi;
  const float b = b2 * m2[i] + ob2 * gi * gi;
  m1[i] = a;
  m2[i] = b;
  const float v = w[i] - lr * (a / c1) / (sqrtf(b / c2) + eps);
  w[i] = v;
  wb[i] = to_bf16(v);
}

unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

struct drot_mlp {
  int device = 0;
  int in = 0, hid = 0, out = 0, max_batch = 0;
  int64_t n_params = 0;
  int64_t off_w[3], off_b[3];  // offsets into the flat parameter vector
  // device buffers
  float* w = nullptr;    // float32 master parameters (flat)
  bf16* wb = nullptr;    // bfloat16 copy
  float* g = nullptr;    // gradients (flat)
  float* m1 = nullptr;
  float* m2 = nullptr;
  float* a[3] = {};  // activations (layer outputs)
  bf16 *ab[3] = {}, *xb = nullptr;
  float* d[3] = {};  // gradients with respect to the pre-activations
  bf16 *db[3] = {};
  double* part = nullptr;
  double* part_host = nullptr;
  float* ksplit = nullptr;  // split-K partial products (kSplitCap floats)
  int64_t step = 0;
};

namespace {

int64_t layer_in(const drot_mlp* n, int l) { return l == 0 ? n->in : n->hid; }
int64_t layer_out(const drot_mlp* n, int l) { return l == 2 ? n->out : n->hid; }

// Split-K workspace: S slices of M x N with S (M / 64) (N / 64) <= 256.
constexpr size_t kSplitCap = (size_t)256 * 64 * 64;

// K slices for an M x N x K product: while the grid has fewer than 256
// workgroups (one per compute unit), halve the depth per workgroup, down to
// 128 (four K steps of 32), up to 8 slices.
int split_k(int M, int N, int K) {
  const int grid = (M / 64) * (N / 64);
  int S = 1;
  while (S < 8 && grid * S * 2 <= 256 && K % (64 * S) == 0 && K / (2 * S) >= 128) S *= 2;
  return S;
}

// One GEMM (see gemm_bf16): epi 0 plain, 1 bias (+ ReLU), 2 ReLU gate; split
// over K (partials in `ws`, then splitk_reduce) when the tile grid alone
// would leave compute units idle.
hipError_t gemm(const bf16* A, const bf16* B, float* C, int M, int N, int K, int lda, int ldb,
                int ldc, int ta, int tb, float beta, hipStream_t s, float* ws, int epi = 0,
                const float* bias = nullptr, const float* gate = nullptr, bf16* Cb = nullptr,
                int relu = 0) {
  const int S = ws ? split_k(M, N, K) : 1;
  const dim3 grid(N / 64, M / 64, S), block(256);
  float* dst = S > 1 ? ws : C;
  const int ldd = S > 1 ? N : ldc;
  const int e = S > 1 ? 3 : epi;
  const int ks = K / S;
#define DROT_GEMM(TA_, TB_, E_)                                                                \
  hipLaunchKernelGGL((gemm_bf16<TA_, TB_, E_>), grid, block, 0, s, A, B, dst, M, N, K, lda, ldb, \
                     ldd, beta, bias, gate, Cb, relu, ks)
  switch (ta * 8 + tb * 4 + e) {
    case 0: DROT_GEMM(0, 0, 0); break;
    case 1: DROT_GEMM(0, 0, 1); break;
    case 2: DROT_GEMM(0, 0, 2); break;
    case 3: DROT_GEMM(0, 0, 3); break;
    case 4: DROT_GEMM(0, 1, 0); break;
    case 5: DROT_GEMM(0, 1, 1); break;
    case 6: DROT_GEMM(0, 1, 2); break;
    case 7: DROT_GEMM(0, 1, 3); break;
    case 8: DROT_GEMM(1, 0, 0); break;
    case 9: DROT_GEMM(1, 0, 1); break;
    case 10: DROT_GEMM(1, 0, 2); break;
    case 11: DROT_GEMM(1, 0, 3); break;
    default: return hipErrorInvalidValue;
  }
#undef DROT_GEMM
  if (S == 1) return hipGetLastError();
  const unsigned nb = (unsigned)(((int64_t)M * N + 255) / 256);
#define DROT_RED(E_)                                                                          \
  hipLaunchKernelGGL((splitk_reduce<E_>), dim3(nb), block, 0, s, ws, S, M, N, C, ldc, beta, bias, \
                     gate, Cb, relu)
  switch (epi) {
    case 0: DROT_RED(0); break;
    case 1: DROT_RED(1); break;
    case 2: DROT_RED(2); break;
    default: return hipErrorInvalidValue;
  }
#undef DROT_RED
  return hipGetLastError();
}

int check_batch(const drot_mlp* n, int batch) {
  if (!n) return mfail(DROT_EINVAL, "mlp is NULL");
  if (batch < 64 || batch % 64 || batch > n->max_batch)
    return mfail(DROT_EINVAL, "batch must be a multiple of 64 in [64, %d]", n->max_batch);
  if (hipSetDevice(n->device) != hipSuccess) return mfail(DROT_EDEVICE, "hipSetDevice failed");
  return DROT_OK;
}

int forward(drot_mlp* n, int B, const float* x, hipStream_t s) {
  hipLaunchKernelGGL(cast_bf16, dim3(nblk((int64_t)B * n->in)), dim3(256), 0, s, x, n->xb,
                     (int64_t)B * n->in);
  MHIP(hipGetLastError());
  const bf16* inp = n->xb;
  for (int l = 0; l < 3; ++l) {
    const int K = (int)layer_in(n, l), N = (int)layer_out(n, l);
    // a_l = act(x_l W_l^T + b_l) and its bfloat16 copy, from the epilogue
    MHIP(gemm(inp, n->wb + n->off_w[l], n->a[l], B, N, K, K, K, N, 0, 1, 0.f, s, n->ksplit, 1,
              n->w + n->off_b[l], nullptr, n->ab[l], l < 2 ? 1 : 0));
    inp = n->ab[l];
  }
  return DROT_OK;
}

// Gradients of the mean-squared error into n->g; loss to *loss (host).
int backward(drot_mlp* n, int B, const float* t, double* loss, hipStream_t s) {
  const int64_t cnt = (int64_t)B * n->out;
  const unsigned nb = nblk(cnt);
  hipLaunchKernelGGL(mse_grad, dim3(nb), dim3(256), 0, s, n->a[2], t, n->d[2], n->db[2], n->part, cnt);
  MHIP(hipGetLastError());
  for (int l = 2; l >= 0; --l) {
    const int K = (int)layer_in(n, l), N = (int)layer_out(n, l);
    const bf16* inp = l == 0 ? n->xb : n->ab[l - 1];
    // dW_l = dZ_l^T x_l  (N x K);  db_l = column sums of dZ_l
    MHIP(gemm(n->db[l], inp, n->g + n->off_w[l], N, K, B, N, K, K, 1, 0, 0.f, s, n->ksplit));
    hipLaunchKernelGGL(col_sum, dim3((N + 63) / 64), dim3(kColSlices * 64), 0, s, n->d[l],
                       n->g + n->off_b[l], B, N);
    MHIP(hipGetLastError());
    if (l > 0) {
      // dZ_{l-1} = (dZ_l W_l) * [a_{l-1} > 0] (B x K), the ReLU gate in the epilogue
      MHIP(gemm(n->db[l], n->wb + n->off_w[l], n->d[l - 1], B, K, N, N, K, K, 0, 0, 0.f, s,
                n->ksplit, 2, nullptr, n->a[l - 1], n->db[l - 1]));
    }
  }
  MHIP(hipMemcpyAsync(n->part_host, n->part, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
  MHIP(hipStreamSynchronize(s));
  double acc = 0.0;
  for (unsigned k = 0; k < nb; ++k) acc += n->part_host[k];
  if (loss) *loss = acc / (double)cnt;
  return DROT_OK;
}

uint64_t splitmix(uint64_t& s) {
  uint64_t z = (s += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

}  // namespace

extern "C" {

int drot_mlp_create(drot_mlp** out, int device, int in, int hidden, int outd, int max_batch,
                    uint64_t seed) {
  if (!out) return mfail(DROT_EINVAL, "out is NULL");
  *out = nullptr;
  if (in < 64 || hidden < 64 || outd < 64 || in % 64 || hidden % 64 || outd % 64)
    return mfail(DROT_EINVAL, "layer widths must be positive multiples of 64");
  if (max_batch < 64 || max_batch % 64) return mfail(DROT_EINVAL, "max_batch must be a multiple of 64");
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
    (void)hipGetLastError();
    return mfail(DROT_EDEVICE, "no HIP device available");
  }
  if (device < 0 || device >= count) return mfail(DROT_EINVAL, "device out of range");
  MHIP(hipSetDevice(device));
  drot_mlp* n = new drot_mlp();
  n->device = device;
  n->in = in;
  n->hid = hidden;
  n->out = outd;
  n->max_batch = max_batch;
  int64_t o = 0;
  for (int l = 0; l < 3; ++l) {
    n->off_w[l] = o;
    o += layer_in(n, l) * layer_out(n, l);
    n->off_b[l] = o;
    o += layer_out(n, l);
  }
  n->n_params = o;
  // He-uniform initialisation from a seeded counter-based generator.
  std::vector<float> hw(o, 0.f);
  uint64_t st = seed;
  for (int l = 0; l < 3; ++l) {
    const double lim = std::sqrt(6.0 / (double)layer_in(n, l));
    for (int64_t k = 0; k < layer_in(n, l) * layer_out(n, l); ++k) {
      const double u = (double)(splitmix(st) >> 11) * (1.0 / 9007199254740992.0);
      hw[n->off_w[l] + k] = (float)((2.0 * u - 1.0) * lim);
    }
  }
  bool ok = hipMalloc(&n->w, sizeof(float) * o) == hipSuccess &&
            hipMalloc(&n->wb, sizeof(bf16) * o) == hipSuccess &&
            hipMalloc(&n->g, sizeof(float) * o) == hipSuccess &&
            hipMalloc(&n->m1, sizeof(float) * o) == hipSuccess &&
            hipMalloc(&n->m2, sizeof(float) * o) == hipSuccess &&
            hipMalloc(&n->xb, sizeof(bf16) * (size_t)max_batch * in) == hipSuccess &&
            hipMalloc(&n->part, sizeof(double) * nblk((int64_t)max_batch * outd)) == hipSuccess &&
            hipMalloc(&n->ksplit, sizeof(float) * kSplitCap) == hipSuccess &&
            hipHostMalloc((void**)&n->part_host, sizeof(double) * nblk((int64_t)max_batch * outd),
                          hipHostMallocDefault) == hipSuccess;
  for (int l = 0; l < 3 && ok; ++l) {
    const size_t c = (size_t)max_batch * layer_out(n, l);
    ok = hipMalloc(&n->a[l], sizeof(float) * c) == hipSuccess &&
         hipMalloc(&n->ab[l], sizeof(bf16) * c) == hipSuccess &&
         hipMalloc(&n->d[l], sizeof(float) * c) == hipSuccess &&
         hipMalloc(&n->db[l], sizeof(bf16) * c) == hipSuccess;
  }
  if (!ok) {
    (void)hipGetLastError();
    drot_mlp_destroy(n);
    return mfail(DROT_ENOMEM, "MLP allocation failed");
  }
  if (drot_mlp_set_weights(n, hw.data()) != DROT_OK) {
    drot_mlp_destroy(n);
    return DROT_EDEVICE;
  }
  *out = n;
  return DROT_OK;
}

int drot_mlp_destroy(drot_mlp* n) {
  if (!n) return DROT_OK;
  (void)hipSetDevice(n->device);
  (void)hipDeviceSynchronize();
  void* bufs[] = {n->w, n->wb, n->g, n->m1, n->m2, n->xb, n->part, n->ksplit};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  for (int l = 0; l < 3; ++l) {
    void* lb[] = {n->a[l], n->ab[l], n->d[l], n->db[l]};
    for (void* b : lb)
      if (b) (void)hipFree(b);
  }
  if (n->part_host) (void)hipHostFree(n->part_host);
  delete n;
  return DROT_OK;
}

int drot_mlp_num_params(const drot_mlp* n, int64_t* count) {
  if (!n || !count) return mfail(DROT_EINVAL, "NULL argument");
  *count = n->n_params;
  return DROT_OK;
}

int drot_mlp_set_weights(drot_mlp* n, const float* host) {
  if (!n || !host) return mfail(DROT_EINVAL, "NULL argument");
  MHIP(hipSetDevice(n->device));
  MHIP(hipMemcpy(n->w, host, sizeof(float) * n->n_params, hipMemcpyHostToDevice));
  hipLaunchKernelGGL(cast_bf16, dim3(nblk(n->n_params)), dim3(256), 0, 0, n->w, n->wb, n->n_params);
  MHIP(hipGetLastError());
  MHIP(hipMemset(n->m1, 0, sizeof(float) * n->n_params));
  MHIP(hipMemset(n->m2, 0, sizeof(float) * n->n_params));
  MHIP(hipDeviceSynchronize());
  n->step = 0;
  return DROT_OK;
}

int drot_mlp_get_weights(drot_mlp* n, float* host) {
  if (!n || !host) return mfail(DROT_EINVAL, "NULL argument");
  MHIP(hipSetDevice(n->device));
  MHIP(hipDeviceSynchronize());
  MHIP(hipMemcpy(host, n->w, sizeof(float) * n->n_params, hipMemcpyDeviceToHost));
  return DROT_OK;
}

int drot_mlp_forward(drot_mlp* n, int batch, const float* x, float* y, void* stream) {
  int rc = check_batch(n, batch);
  if (rc) return rc;
  if (!x || !y) return mfail(DROT_EINVAL, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  if ((rc = forward(n, batch, x, s))) return rc;
  MHIP(hipMemcpyAsync(y, n->a[2], sizeof(float) * (size_t)batch * n->out, hipMemcpyDeviceToDevice, s));
  return DROT_OK;
}

int drot_mlp_gradients(drot_mlp* n, int batch, const float* x, const float* t, float* grad,
                       double* loss, void* stream) {
  int rc = check_batch(n, batch);
  if (rc) return rc;
  if (!x || !t) return mfail(DROT_EINVAL, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  if ((rc = forward(n, batch, x, s))) return rc;
  if ((rc = backward(n, batch, t, loss, s))) return rc;
  if (grad) MHIP(hipMemcpyAsync(grad, n->g, sizeof(float) * n->n_params, hipMemcpyDeviceToDevice, s));
  return DROT_OK;
}

}  // extern "C"

namespace {

// One Adam step with the gradient in `g` (device, flat parameter order).
int adam_step(drot_mlp* n, const float* g, float lr, hipStream_t s) {
  n->step += 1;
  const double b1 = 0.9, b2 = 0.999;
  const double c1 = 1.0 - std::pow(b1, (double)n->step), c2 = 1.0 - std::pow(b2, (double)n->step);
  hipLaunchKernelGGL(adam, dim3(nblk(n->n_params)), dim3(256), 0, s, n->w, n->wb, g, n->m1,
                     n->m2, n->n_params, lr, (float)b1, (float)(1.0 - b1), (float)b2,
                     (float)(1.0 - b2), 1e-8f, (float)c1, (float)c2);
  MHIP(hipGetLastError());
  return DROT_OK;
}

}  // namespace

extern "C" {

int drot_mlp_train_step(drot_mlp* n, int batch, const float* x, const float* t, float lr,
                        double* loss, void* stream) {
  if (!(lr > 0.f)) return mfail(DROT_EINVAL, "lr must be positive");
  int rc = drot_mlp_gradients(n, batch, x, t, nullptr, loss, stream);
  if (rc) return rc;
  return adam_step(n, n->g, lr, (hipStream_t)stream);
}

int drot_mlp_apply_gradients(drot_mlp* n, const float* grad, float lr, void* stream) {
  if (!n || !grad) return mfail(DROT_EINVAL, "NULL argument");
  if (!(lr > 0.f)) return mfail(DROT_EINVAL, "lr must be positive");
  MHIP(hipSetDevice(n->device));
  return adam_step(n, grad, lr, (hipStream_t)stream);
}

}  // extern "C"

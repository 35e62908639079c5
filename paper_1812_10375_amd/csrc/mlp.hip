// mlp.hip -- boiling-curve surrogate: ensemble of 4 -> 128 -> 128 -> 2 GELU MLPs with
// BF16 matrix-core products (FP32 accumulation), backward pass and Adam.
//
// Every layer product, forward and backward, is one launch of k_gemm_bf16: a wave
// owns a 16 x 16 output tile and runs v_mfma_f32_16x16x32_bf16 down the contraction,
// operands addressed through (row, column) strides so that transposed views cost
// nothing; an epilogue applies the bias and GELU (forward) or the GELU derivative
// (backward) and writes FP32 and/or BF16 results.  Padding: layer 1 contracts over 32
// (inputs 4..31 are zero), layer 3 produces 16 columns (outputs 2..15 have zero weights).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "lbm_api.h"
#include "lbm_mlp.h"

namespace {

constexpr int IN = LBM_MLP_IN, H = LBM_MLP_HIDDEN, OUT = LBM_MLP_OUT;
constexpr int KP1 = 32, NP3 = 16;  // padded contraction of layer 1, padded width of layer 3
// padded parameter block of one member (floats)
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + KP1 * H, OFF_W2 = OFF_B1 + H, OFF_B2 = OFF_W2 + H * H,
              OFF_W3 = OFF_B2 + H, OFF_B3 = OFF_W3 + H * NP3, PP = OFF_B3 + NP3;
// host parameter block of one member (floats)
constexpr int HP = IN * H + H + H * H + H + H * OUT + OUT;
constexpr int MAX_MEMBERS = 16, MAX_BATCH = 1 << 20;

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

enum { EPI_F32 = 0, EPI_BIAS_GELU = 1, EPI_BIAS_OUT = 2, EPI_GELU_GRAD = 3, EPI_BIAS_GELU_BF16 = 4 };

struct Gemm {
  const __bf16* A;  // A(m, k) = A[m * sam + k * sak + z * saz]
  long sam, sak, saz;
  const __bf16* B;  // B(k, n) = B[k * sbk + n * sbn + z * sbz]
  long sbk, sbn, sbz;
  int M, N, K;
  const float* bias;  // bias[n + z * sbias]
  long sbias;
  float* Cf;  // FP32 result [m * ldc + n + z * scf]
  long ldc, scf;
  __bf16* Cb;  // BF16 result [m * ldb + n + z * scb]
  long ldb, scb;
  const float* Zin;  // pre-activation for the GELU derivative [m * ldz + n + z * szz]
  long ldz, szz;
  int nvalid;  // columns written by EPI_BIAS_OUT
  const float* Dsum;  // split-K only: blocks of the first tile row also sum the columns of
  float* dbias;       // Dsum ([K][N] per member, stride sdsum) into dbias (stride sdbias)
  long sdsum, sdbias;
};

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float z) {
  return 0.5f * (1.f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

// C = A B over a 16 x 16 tile per wave, 4 waves per block, blockIdx.y = ensemble member.
// Matrix-core lane layout (16x16x32): lane l feeds row (l & 15) of A and column (l & 15)
// of B with 8 contraction indices starting at 8 (l >> 4), and receives rows
// 4 (l >> 4) + r (r = 0..3) of column (l & 15) of the result.
template <int EPI>
__global__ void __launch_bounds__(256) k_gemm_bf16(const Gemm g) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int z = blockIdx.y;
  const int tn = (g.N + 15) / 16, tm = (g.M + 15) / 16;
  const int tile = blockIdx.x * 4 + wave;
  if (tile >= tm * tn) return;  // whole wave
  const int m0 = (tile / tn) * 16, n0 = (tile % tn) * 16;
  const int i = lane & 15, kq = lane >> 4;
  const __bf16* A = g.A + z * g.saz;
  const __bf16* B = g.B + z * g.sbz;
  const bool row_ok = m0 + i < g.M, col_ok = n0 + i < g.N;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < g.K; k0 += 32) {
    bf16x8 a, b;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = k0 + 8 * kq + e;
      const bool k_ok = k < g.K;
      a[e] = (row_ok && k_ok) ? A[(long)(m0 + i) * g.sam + (long)k * g.sak] : (__bf16)0.f;
      b[e] = (col_ok && k_ok) ? B[(long)k * g.sbk + (long)(n0 + i) * g.sbn] : (__bf16)0.f;
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
  }
  const int n = n0 + i;
  if (n >= g.N) return;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int m = m0 + 4 * kq + r;
    if (m >= g.M) continue;
    const float v = acc[r];
    if constexpr (EPI == EPI_F32) {
      g.Cf[(long)m * g.ldc + n + z * g.scf] = v;
    } else if constexpr (EPI == EPI_BIAS_GELU) {
      const float zz = v + g.bias[n + z * g.sbias];
      g.Cf[(long)m * g.ldc + n + z * g.scf] = zz;
      g.Cb[(long)m * g.ldb + n + z * g.scb] = (__bf16)gelu(zz);
    } else if constexpr (EPI == EPI_BIAS_GELU_BF16) {
      // inference only: the BF16 activation, without the FP32 pre-activation
      g.Cb[(long)m * g.ldb + n + z * g.scb] = (__bf16)gelu(v + g.bias[n + z * g.sbias]);
    } else if constexpr (EPI == EPI_BIAS_OUT) {
      if (n < g.nvalid) g.Cf[(long)m * g.ldc + n + z * g.scf] = v + g.bias[n + z * g.sbias];
    } else {
      const float d = v * gelu_grad(g.Zin[(long)m * g.ldz + n + z * g.szz]);
      g.Cf[(long)m * g.ldc + n + z * g.scf] = d;
      g.Cb[(long)m * g.ldb + n + z * g.scb] = (__bf16)d;
    }
  }
}

// db[n] = sum over rows of D[row][n] for the 16 columns n0 .. n0 + 15 (n < N, row < B),
// in a fixed order, by a block of 1024 threads: thread (g, c) sums rows g, g + 64, ...
// of column n0 + c in order, and the 64 row-group partials are added pairwise in LDS.
// Every thread of the block must call it.
constexpr int CS_THREADS = 1024, CS_COLS = 16, CS_GROUPS = CS_THREADS / CS_COLS;
__device__ __forceinline__ void colsum16(const float* __restrict__ D, int B, int N, int n0, float* __restrict__ db) {
  __shared__ float part[CS_GROUPS][CS_COLS];
  const int c = threadIdx.x % CS_COLS, grp = threadIdx.x / CS_COLS;
  const int n = n0 + c;
  float s = 0.f;
  if (n < N)
    for (int b = grp; b < B; b += CS_GROUPS) s += D[(long)b * N + n];
  part[grp][c] = s;
  __syncthreads();
  for (int h = CS_GROUPS / 2; h > 0; h >>= 1) {
    if (grp < h) part[grp][c] += part[grp + h][c];
    __syncthreads();
  }
  if (grp == 0 && n < N) db[n] = part[0][c];
}

// The weight-gradient products contract over the batch (K = B rows) into few output
// tiles.  Here the 16 waves of a block share one 16 x 16 tile: wave w takes the k-steps
// w, w + 16, ... of 32, and lane l of wave 0 adds the 16 partial tiles in wave order.
constexpr int SK_WAVES = 16;
__global__ void __launch_bounds__(SK_WAVES * 64) k_gemm_bf16_splitk(const Gemm g) {
  __shared__ f32x4 part[SK_WAVES][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int z = blockIdx.y;
  const int tn = (g.N + 15) / 16;
  const int tile = blockIdx.x;
  const int m0 = (tile / tn) * 16, n0 = (tile % tn) * 16;
  const int i = lane & 15, kq = lane >> 4;
  const __bf16* A = g.A + z * g.saz;
  const __bf16* B = g.B + z * g.sbz;
  const bool row_ok = m0 + i < g.M, col_ok = n0 + i < g.N;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 32 * wave; k0 < g.K; k0 += 32 * SK_WAVES) {
    bf16x8 a, b;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = k0 + 8 * kq + e;
      const bool k_ok = k < g.K;
      a[e] = (row_ok && k_ok) ? A[(long)(m0 + i) * g.sam + (long)k * g.sak] : (__bf16)0.f;
      b[e] = (col_ok && k_ok) ? B[(long)k * g.sbk + (long)(n0 + i) * g.sbn] : (__bf16)0.f;
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
  }
  if (g.dbias && m0 == 0) colsum16(g.Dsum + z * g.sdsum, g.K, g.N, n0, g.dbias + z * g.sdbias);
  part[wave][lane] = acc;
  __syncthreads();
  if (wave != 0) return;
  f32x4 t = part[0][lane];
  for (int q = 1; q < SK_WAVES; ++q) t += part[q][lane];
  const int n = n0 + i;
  if (n >= g.N) return;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int m = m0 + 4 * kq + r;
    if (m < g.M) g.Cf[(long)m * g.ldc + n + z * g.scf] = t[r];
  }
}

// inputs [B][4] FP32 (member z at x + z * sx) -> [B][32] BF16 (member z at xb + z * sxb),
// zero beyond column 4; blockIdx.y = member
__global__ void k_prep_x(const float* __restrict__ x, long sx, __bf16* __restrict__ xb, long sxb, int B) {
  const int z = blockIdx.y;
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < (long)B * KP1; t += (long)gridDim.x * blockDim.x) {
    const int c = (int)(t % KP1);
    const long b = t / KP1;
    xb[z * sxb + t] = (__bf16)(c < IN ? x[z * sx + b * IN + c] : 0.f);
  }
}


// dY = 2 (Y - T) / B on the 2 outputs (zero on the padded columns), and the loss of
// each member: one block per member, fixed-order reduction.
constexpr int OG_THREADS = 1024;
__global__ void __launch_bounds__(OG_THREADS) k_out_grad(const float* __restrict__ Y, const float* __restrict__ T, long st,
                                                   int B, float* __restrict__ dYf, __bf16* __restrict__ dYb,
                                                   float* __restrict__ loss, long sy, long sd,
                                                   float* __restrict__ db3, long sdb) {
  __shared__ float red[OG_THREADS];
  const int z = blockIdx.x;
  const float inv = 1.f / (float)B;
  float acc = 0.f;
  for (long t = threadIdx.x; t < (long)B * NP3; t += OG_THREADS) {
    const long b = t / NP3;
    const int c = (int)(t % NP3);
    float d = 0.f;
    if (c < OUT) {
      const float e = Y[z * sy + b * OUT + c] - T[z * st + b * OUT + c];
      acc += e * e;
      d = 2.f * e * inv;
    }
    dYf[z * sd + t] = d;
    dYb[z * sd + t] = (__bf16)d;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = OG_THREADS / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[z] = red[0] * inv;
  // bias gradient of the output layer: the column sums of dY
  colsum16(dYf + z * sd, B, NP3, 0, db3 + z * sdb);
}

__global__ void k_to_bf16(const float* __restrict__ w, __bf16* __restrict__ wb, long n) {
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x)
    wb[t] = (__bf16)w[t];
}

__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m1,
                       float* __restrict__ m2, __bf16* __restrict__ wb, long n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
    const float gg = g[t];
    const float a = b1 * m1[t] + (1.f - b1) * gg;
    const float v = b2 * m2[t] + (1.f - b2) * gg * gg;
    m1[t] = a;
    m2[t] = v;
    const float wn = w[t] - lr * (a * c1) / (sqrtf(v * c2) + eps);
    w[t] = wn;
    wb[t] = (__bf16)wn;
  }
}

size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

struct Layout {
  size_t w, g, m1, m2, wb, xb, z1, h1, z2, h2, y, dyf, dyb, d2f, d2b, d1f, d1b, total;
};

Layout layout(int M, int Bm) {
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  const size_t P = (size_t)M * PP, A = (size_t)M * Bm;
  L.w = take(P * 4);
  L.g = take(P * 4);
  L.m1 = take(P * 4);
  L.m2 = take(P * 4);
  L.wb = take(P * 2);
  L.xb = take(A * KP1 * 2);
  L.z1 = take(A * H * 4);
  L.h1 = take(A * H * 2);
  L.z2 = take(A * H * 4);
  L.h2 = take(A * H * 2);
  L.y = take(A * OUT * 4);
  L.dyf = take(A * NP3 * 4);
  L.dyb = take(A * NP3 * 2);
  L.d2f = take(A * H * 4);
  L.d2b = take(A * H * 2);
  L.d1f = take(A * H * 4);
  L.d1b = take(A * H * 2);
  L.total = off;
  return L;
}

}  // namespace

struct lbm_mlp {
  int members, max_batch;
  int device;  // device current at init
  hipStream_t stream;
  char* ws;
  Layout L;
  long step;
  template <typename T>
  T* at(size_t off) const {
    return reinterpret_cast<T*>(ws + off);
  }
};

namespace {

int hip_rc(hipError_t e) { return e == hipSuccess ? LBM_OK : LBM_EHIP; }

template <int EPI>
void gemm(lbm_mlp* m, const Gemm& g) {
  const int tiles = ((g.M + 15) / 16) * ((g.N + 15) / 16);
  // long contractions into few tiles are split over K; so are those that also sum
  // bias-gradient columns, which the split kernel does in its first tile row
  if (EPI == EPI_F32 && (g.K >= 32 * SK_WAVES || g.dbias))
    hipLaunchKernelGGL(k_gemm_bf16_splitk, dim3(tiles, m->members), dim3(SK_WAVES * 64), 0, m->stream, g);
  else
    hipLaunchKernelGGL(k_gemm_bf16<EPI>, dim3((tiles + 3) / 4, m->members), dim3(256), 0, m->stream, g);
}

Gemm blank() {
  Gemm g;
  std::memset(&g, 0, sizeof(g));
  return g;
}

// forward pass of every member: Z1, H1, Z2, H2 into the workspace, outputs to y
// ([members][B][2] with member stride sy)
void forward(lbm_mlp* m, const float* x, long sx, int B, float* y, long sy) {
  const Layout& L = m->L;
  const long A = (long)m->max_batch;  // member stride of the activation arrays, in rows
  hipLaunchKernelGGL(k_prep_x, dim3(256, m->members), dim3(256), 0, m->stream, x, sx, m->at<__bf16>(L.xb), A * KP1,
                     B);
  const __bf16* wb = m->at<__bf16>(L.wb);
  const float* w = m->at<float>(L.w);
  Gemm g = blank();
  // layer 1: Z1 = X W1 + b1, H1 = gelu(Z1)
  g.A = m->at<__bf16>(L.xb); g.sam = KP1; g.sak = 1; g.saz = A * KP1;
  g.B = wb + OFF_W1; g.sbk = H; g.sbn = 1; g.sbz = PP;
  g.M = B; g.N = H; g.K = KP1;
  g.bias = w + OFF_B1; g.sbias = PP;
  g.Cf = m->at<float>(L.z1); g.ldc = H; g.scf = A * H;
  g.Cb = m->at<__bf16>(L.h1); g.ldb = H; g.scb = A * H;
  gemm<EPI_BIAS_GELU>(m, g);
  // layer 2: Z2 = H1 W2 + b2, H2 = gelu(Z2)
  g = blank();
  g.A = m->at<__bf16>(L.h1); g.sam = H; g.sak = 1; g.saz = A * H;
  g.B = wb + OFF_W2; g.sbk = H; g.sbn = 1; g.sbz = PP;
  g.M = B; g.N = H; g.K = H;
  g.bias = w + OFF_B2; g.sbias = PP;
  g.Cf = m->at<float>(L.z2); g.ldc = H; g.scf = A * H;
  g.Cb = m->at<__bf16>(L.h2); g.ldb = H; g.scb = A * H;
  gemm<EPI_BIAS_GELU>(m, g);
  // layer 3: Y = H2 W3 + b3 (2 of the 16 padded columns)
  g = blank();
  g.A = m->at<__bf16>(L.h2); g.sam = H; g.sak = 1; g.saz = A * H;
  g.B = wb + OFF_W3; g.sbk = NP3; g.sbn = 1; g.sbz = PP;
  g.M = B; g.N = NP3; g.K = H;
  g.bias = w + OFF_B3; g.sbias = PP;
  g.Cf = y; g.ldc = OUT; g.scf = sy;
  g.nvalid = OUT;
  gemm<EPI_BIAS_OUT>(m, g);
}

// Activations of the allocation-free forward pass: one file-scope device array, held
// by every device the library runs on until the process ends.  Per row (a member's
// input row): padded BF16 inputs (32), then the BF16 activations of both hidden layers
// (128 each).  Host code reaches it only through the device address that
// hipGetSymbolAddress returns on each device.
constexpr long NOALLOC_ROWS = LBM_MLP_NOALLOC_MAX_ROWS;
constexpr size_t NA_XB = 0, NA_H1 = NA_XB + (size_t)NOALLOC_ROWS * KP1 * 2,
                 NA_H2 = NA_H1 + (size_t)NOALLOC_ROWS * H * 2, NA_BYTES = NA_H2 + (size_t)NOALLOC_ROWS * H * 2;
static_assert(NA_H1 % 256 == 0 && NA_H2 % 256 == 0, "scratch parts stay 256-byte aligned");
static __device__ __align__(256) unsigned char scratch[NA_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
char* scratch_dev[MAX_DEVICES];  // device address of `scratch` on each device, once resolved

// Resolve the device address of `scratch` on the current device (once per device).
int resolve_scratch(int& device) {
  if (hipGetDevice(&device) != hipSuccess || device < 0 || device >= MAX_DEVICES) return LBM_EHIP;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_dev[device]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return LBM_EHIP;
    scratch_dev[device] = static_cast<char*>(ptr);
  }
  return LBM_OK;
}

// The forward pass of every member with its activations in `sc` (the device address of
// `scratch`): the same kernels, operands and accumulation order as forward(), so the
// outputs are identical; only the FP32 pre-activations are not kept.
void forward_scratch(lbm_mlp* m, char* sc, const float* x, int B, float* y) {
  const long A = (long)B;  // member stride in rows
  __bf16* xb = reinterpret_cast<__bf16*>(sc + NA_XB);
  __bf16* h1 = reinterpret_cast<__bf16*>(sc + NA_H1);
  __bf16* h2 = reinterpret_cast<__bf16*>(sc + NA_H2);
  hipLaunchKernelGGL(k_prep_x, dim3(256, m->members), dim3(256), 0, m->stream, x, 0L, xb, A * KP1, B);
  const __bf16* wb = m->at<__bf16>(m->L.wb);
  const float* w = m->at<float>(m->L.w);
  Gemm g = blank();
  g.A = xb; g.sam = KP1; g.sak = 1; g.saz = A * KP1;
  g.B = wb + OFF_W1; g.sbk = H; g.sbn = 1; g.sbz = PP;
  g.M = B; g.N = H; g.K = KP1;
  g.bias = w + OFF_B1; g.sbias = PP;
  g.Cb = h1; g.ldb = H; g.scb = A * H;
  gemm<EPI_BIAS_GELU_BF16>(m, g);
  g = blank();
  g.A = h1; g.sam = H; g.sak = 1; g.saz = A * H;
  g.B = wb + OFF_W2; g.sbk = H; g.sbn = 1; g.sbz = PP;
  g.M = B; g.N = H; g.K = H;
  g.bias = w + OFF_B2; g.sbias = PP;
  g.Cb = h2; g.ldb = H; g.scb = A * H;
  gemm<EPI_BIAS_GELU_BF16>(m, g);
  g = blank();
  g.A = h2; g.sam = H; g.sak = 1; g.saz = A * H;
  g.B = wb + OFF_W3; g.sbk = NP3; g.sbn = 1; g.sbz = PP;
  g.M = B; g.N = NP3; g.K = H;
  g.bias = w + OFF_B3; g.sbias = PP;
  g.Cf = y; g.ldc = OUT; g.scf = (long)B * OUT;
  g.nvalid = OUT;
  gemm<EPI_BIAS_OUT>(m, g);
}

bool valid_sizes(int members, int max_batch) {
  return members >= 1 && members <= MAX_MEMBERS && max_batch >= 1 && max_batch <= MAX_BATCH;
}

}  // namespace

extern "C" {

size_t lbm_mlp_params(void) { return HP; }

size_t lbm_mlp_workspace_bytes(int members, int max_batch) {
  if (!valid_sizes(members, max_batch)) return 0;
  return layout(members, max_batch).total;
}

int lbm_mlp_init(int members, int max_batch, void* d_workspace, size_t ws_bytes, void* hip_stream,
                 lbm_mlp** out) {
  if (!out) return LBM_EINVAL;
  *out = nullptr;
  if (!valid_sizes(members, max_batch) || !d_workspace) return LBM_EINVAL;
  if (reinterpret_cast<uintptr_t>(d_workspace) & 255) return LBM_EINVAL;
  const Layout L = layout(members, max_batch);
  if (ws_bytes < L.total) return LBM_ENOMEM;
  int device = -1;
  if (resolve_scratch(device) != LBM_OK) return LBM_EHIP;
  lbm_mlp* m = new (std::nothrow) lbm_mlp();
  if (!m) return LBM_ENOMEM;
  m->device = device;
  m->members = members;
  m->max_batch = max_batch;
  m->stream = reinterpret_cast<hipStream_t>(hip_stream);
  m->ws = reinterpret_cast<char*>(d_workspace);
  m->L = L;
  m->step = 0;
  // parameters, gradients, moments and BF16 copies start at zero
  const size_t zero_bytes = L.xb;
  if (hipMemsetAsync(m->ws, 0, zero_bytes, m->stream) != hipSuccess ||
      hipStreamSynchronize(m->stream) != hipSuccess) {
    delete m;
    return LBM_EHIP;
  }
  *out = m;
  return LBM_OK;
}

int lbm_mlp_set_params(lbm_mlp* m, const float* host) {
  if (!m || !host) return LBM_EINVAL;
  std::vector<float> pad((size_t)m->members * PP, 0.f);
  for (int z = 0; z < m->members; ++z) {
    const float* s = host + (size_t)z * HP;
    float* d = pad.data() + (size_t)z * PP;
    for (int k = 0; k < IN; ++k)
      for (int n = 0; n < H; ++n) d[OFF_W1 + k * H + n] = s[k * H + n];
    s += IN * H;
    for (int n = 0; n < H; ++n) d[OFF_B1 + n] = s[n];
    s += H;
    for (int k = 0; k < H * H; ++k) d[OFF_W2 + k] = s[k];
    s += H * H;
    for (int n = 0; n < H; ++n) d[OFF_B2 + n] = s[n];
    s += H;
    for (int k = 0; k < H; ++k)
      for (int n = 0; n < OUT; ++n) d[OFF_W3 + k * NP3 + n] = s[k * OUT + n];
    s += H * OUT;
    for (int n = 0; n < OUT; ++n) d[OFF_B3 + n] = s[n];
  }
  const Layout& L = m->L;
  const size_t bytes = pad.size() * 4;
  int rc = hip_rc(hipMemcpyAsync(m->at<float>(L.w), pad.data(), bytes, hipMemcpyHostToDevice, m->stream));
  if (!rc) rc = hip_rc(hipMemsetAsync(m->at<float>(L.m1), 0, bytes, m->stream));
  if (!rc) rc = hip_rc(hipMemsetAsync(m->at<float>(L.m2), 0, bytes, m->stream));
  if (rc) return rc;
  hipLaunchKernelGGL(k_to_bf16, dim3(128), dim3(256), 0, m->stream, m->at<float>(L.w), m->at<__bf16>(L.wb),
                     (long)pad.size());
  m->step = 0;
  rc = hip_rc(hipGetLastError());
  if (!rc) rc = hip_rc(hipStreamSynchronize(m->stream));  // `pad` is freed on return
  return rc;
}

static int copy_out(lbm_mlp* m, size_t off, float* host) {
  std::vector<float> pad((size_t)m->members * PP);
  int rc = hip_rc(hipMemcpyAsync(pad.data(), m->at<float>(off), pad.size() * 4, hipMemcpyDeviceToHost, m->stream));
  if (!rc) rc = hip_rc(hipStreamSynchronize(m->stream));
  if (rc) return rc;
  for (int z = 0; z < m->members; ++z) {
    const float* s = pad.data() + (size_t)z * PP;
    float* d = host + (size_t)z * HP;
    for (int k = 0; k < IN; ++k)
      for (int n = 0; n < H; ++n) *d++ = s[OFF_W1 + k * H + n];
    for (int n = 0; n < H; ++n) *d++ = s[OFF_B1 + n];
    for (int k = 0; k < H * H; ++k) *d++ = s[OFF_W2 + k];
    for (int n = 0; n < H; ++n) *d++ = s[OFF_B2 + n];
    for (int k = 0; k < H; ++k)
      for (int n = 0; n < OUT; ++n) *d++ = s[OFF_W3 + k * NP3 + n];
    for (int n = 0; n < OUT; ++n) *d++ = s[OFF_B3 + n];
  }
  return LBM_OK;
}

int lbm_mlp_get_params(lbm_mlp* m, float* host) {
  if (!m || !host) return LBM_EINVAL;
  return copy_out(m, m->L.w, host);
}

int lbm_mlp_get_grads(lbm_mlp* m, float* host) {
  if (!m || !host) return LBM_EINVAL;
  return copy_out(m, m->L.g, host);
}

int lbm_mlp_forward(lbm_mlp* m, const float* d_x, int B, float* d_y) {
  if (!m || !d_x || !d_y || B < 1 || B > m->max_batch) return LBM_EINVAL;
  forward(m, d_x, 0, B, d_y, (long)B * OUT);
  return hip_rc(hipGetLastError());
}

int lbm_mlp_forward_noalloc(lbm_mlp* m, const float* d_x, int B, float* d_y) {
  if (!m || !d_x || !d_y || B < 1 || (long)m->members * B > NOALLOC_ROWS) return LBM_EINVAL;
  char* sc = (m->device >= 0 && m->device < MAX_DEVICES) ? scratch_dev[m->device] : nullptr;
  if (!sc) return LBM_EHIP;
  forward_scratch(m, sc, d_x, B, d_y);
  return hip_rc(hipGetLastError());
}

int lbm_mlp_backward(lbm_mlp* m, const float* d_x, const float* d_t, int B, int per_member, float* d_loss) {
  if (!m || !d_x || !d_t || !d_loss || B < 1 || B > m->max_batch) return LBM_EINVAL;
  const Layout& L = m->L;
  const long A = (long)m->max_batch;
  float* Y = m->at<float>(L.y);
  const long sx = per_member ? (long)B * IN : 0, st = per_member ? (long)B * OUT : 0;
  forward(m, d_x, sx, B, Y, A * OUT);
  float* gr = m->at<float>(L.g);
  hipLaunchKernelGGL(k_out_grad, dim3(m->members), dim3(OG_THREADS), 0, m->stream, Y, d_t, st, B, m->at<float>(L.dyf),
                     m->at<__bf16>(L.dyb), d_loss, A * OUT, A * NP3, gr + OFF_B3, (long)PP);
  const __bf16* wb = m->at<__bf16>(L.wb);
  Gemm g = blank();
  // dW3 = H2^T dY (128 x 16)
  g.A = m->at<__bf16>(L.h2); g.sam = 1; g.sak = H; g.saz = A * H;
  g.B = m->at<__bf16>(L.dyb); g.sbk = NP3; g.sbn = 1; g.sbz = A * NP3;
  g.M = H; g.N = NP3; g.K = B;
  g.Cf = gr + OFF_W3; g.ldc = NP3; g.scf = PP;
  gemm<EPI_F32>(m, g);
  // dZ2 = (dY W3^T) * gelu'(Z2)
  g = blank();
  g.A = m->at<__bf16>(L.dyb); g.sam = NP3; g.sak = 1; g.saz = A * NP3;
  g.B = wb + OFF_W3; g.sbk = 1; g.sbn = NP3; g.sbz = PP;
  g.M = B; g.N = H; g.K = NP3;
  g.Zin = m->at<float>(L.z2); g.ldz = H; g.szz = A * H;
  g.Cf = m->at<float>(L.d2f); g.ldc = H; g.scf = A * H;
  g.Cb = m->at<__bf16>(L.d2b); g.ldb = H; g.scb = A * H;
  gemm<EPI_GELU_GRAD>(m, g);
  // dW2 = H1^T dZ2 (128 x 128)
  g = blank();
  g.A = m->at<__bf16>(L.h1); g.sam = 1; g.sak = H; g.saz = A * H;
  g.B = m->at<__bf16>(L.d2b); g.sbk = H; g.sbn = 1; g.sbz = A * H;
  g.M = H; g.N = H; g.K = B;
  g.Cf = gr + OFF_W2; g.ldc = H; g.scf = PP;
  g.Dsum = m->at<float>(L.d2f); g.sdsum = A * H; g.dbias = gr + OFF_B2; g.sdbias = PP;  // db2 = column sums of dZ2
  gemm<EPI_F32>(m, g);
  // dZ1 = (dZ2 W2^T) * gelu'(Z1)
  g = blank();
  g.A = m->at<__bf16>(L.d2b); g.sam = H; g.sak = 1; g.saz = A * H;
  g.B = wb + OFF_W2; g.sbk = 1; g.sbn = H; g.sbz = PP;
  g.M = B; g.N = H; g.K = H;
  g.Zin = m->at<float>(L.z1); g.ldz = H; g.szz = A * H;
  g.Cf = m->at<float>(L.d1f); g.ldc = H; g.scf = A * H;
  g.Cb = m->at<__bf16>(L.d1b); g.ldb = H; g.scb = A * H;
  gemm<EPI_GELU_GRAD>(m, g);
  // dW1 = X^T dZ1 (32 x 128; rows 4..31 are zero since the padded inputs are)
  g = blank();
  g.A = m->at<__bf16>(L.xb); g.sam = 1; g.sak = KP1; g.saz = A * KP1;
  g.B = m->at<__bf16>(L.d1b); g.sbk = H; g.sbn = 1; g.sbz = A * H;
  g.M = KP1; g.N = H; g.K = B;
  g.Cf = gr + OFF_W1; g.ldc = H; g.scf = PP;
  g.Dsum = m->at<float>(L.d1f); g.sdsum = A * H; g.dbias = gr + OFF_B1; g.sdbias = PP;  // db1 = column sums of dZ1
  gemm<EPI_F32>(m, g);
  return hip_rc(hipGetLastError());
}

int lbm_mlp_adam(lbm_mlp* m, float lr, float beta1, float beta2, float eps) {
  if (!m || !(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return LBM_EINVAL;
  const Layout& L = m->L;
  m->step += 1;
  const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, (double)m->step)));
  const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, (double)m->step)));
  hipLaunchKernelGGL(k_adam, dim3(256), dim3(256), 0, m->stream, m->at<float>(L.w), m->at<float>(L.g),
                     m->at<float>(L.m1), m->at<float>(L.m2), m->at<__bf16>(L.wb), (long)m->members * PP, lr,
                     beta1, beta2, eps, c1, c2);
  return hip_rc(hipGetLastError());
}

int lbm_mlp_destroy(lbm_mlp* m) {
  if (!m) return LBM_EINVAL;
  delete m;
  return LBM_OK;
}

}  // extern "C"

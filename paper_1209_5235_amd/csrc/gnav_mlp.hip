// gnav_mlp.hip -- training kernels of the candidate-ordering MLP (bf16 MFMA,
// float32 accumulation) and their C ABI.
//
// The network scores the candidates of a voxel node during ComputeStep:
// inputs are the point and direction in the mother frame (6 values) and the
// mother volume (a class id, realised as a row gather of the first layer's
// weights); two hidden layers of 128 ReLU units; 64 logits, one per candidate
// position.  Training data are crossings recorded by the transport itself.
//
// Matrix products use v_mfma_f32_16x16x16_bf16: each wave computes one 16x16
// output tile, K in steps of 16.  Operand layout per lane l (wave64):
//   A (16 x 16, rows m, columns k): row m = l % 16, k = 4 (l / 16) + 0..3
//   B (16 x 16, rows k, columns n): column n = l % 16, k = 4 (l / 16) + 0..3
//   D (16 x 16 float):              column n = l % 16, rows 4 (l / 16) + 0..3
// Element-wise work (bias, ReLU, masks, casts, softmax) runs on the VALU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "gnav.h"
#include "gnav_internal.h"

namespace gnav {

constexpr int kNIn = 6, kNH = 128, kNOut = 64;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float32 -> bfloat16 bits, round to nearest even (NaN kept quiet).
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

// C[m][n] = sum_k A(m, k) B(k, n); A(m, k) = A[m * sam + k * sak], B(k, n) =
// B[k * sbk + n * sbn] (bf16 bits), C float with row stride ldc.  M, N, K are
// multiples of 16.  One wave per 16x16 tile; grid.x covers all tiles.  With
// grid.y > 1 the sum over k is split: slice y covers k in [y kc, (y+1) kc) and
// writes its partial product to C + y cstride (kc a multiple of 16).
__global__ void __launch_bounds__(256) k_gemm_bf16(int M, int N, int K, int kc, const uint16_t* __restrict__ A,
                                                   long sam, long sak, const uint16_t* __restrict__ B,
                                                   long sbk, long sbn, float* __restrict__ C, long ldc,
                                                   long cstride) {
  const int lane = threadIdx.x & 63;
  const long tile = (long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int tn = N / 16;
  const long tiles = (long)(M / 16) * tn;
  if (tile >= tiles) return;
  const int m0 = (int)(tile / tn) * 16, n0 = (int)(tile % tn) * 16;
  const int r = lane & 15, q = lane >> 4;
  const int kb = (int)blockIdx.y * kc, ke = min(K, kb + kc);
  C += (long)blockIdx.y * cstride;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = kb; k0 < ke; k0 += 16) {
    bf16x4 a, b;
#pragma unroll
    for (int j = 0; j < 4; j++) {
      int k = k0 + 4 * q + j;
      a[j] = (short)A[(long)(m0 + r) * sam + (long)k * sak];
      b[j] = (short)B[(long)k * sbk + (long)(n0 + r) * sbn];
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int j = 0; j < 4; j++) C[(long)(m0 + 4 * q + j) * ldc + (n0 + r)] = acc[j];
}

__global__ void k_cast_bf16(const float* __restrict__ src, uint16_t* __restrict__ dst, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    dst[i] = f2bf(src[i]);
}

// Layer 1: A1 = bf16(x) W1x^T + W1m[cls] + b1 (float), H1b = bf16(ReLU(A1)).
__global__ void k_layer1(int B, const float* __restrict__ x, const int* __restrict__ cls, int n_class,
                         const uint16_t* __restrict__ w1x, const uint16_t* __restrict__ w1m,
                         const float* __restrict__ b1, uint16_t* __restrict__ xb, float* __restrict__ a1,
                         uint16_t* __restrict__ h1b) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)B * kNH) return;
  int b = (int)(i / kNH), h = (int)(i % kNH);
  float acc = 0.f;
#pragma unroll
  for (int k = 0; k < kNIn; k++) acc += bf2f(f2bf(x[b * kNIn + k])) * bf2f(w1x[h * kNIn + k]);
  int c = cls[b];
  c = c < 0 ? 0 : (c >= n_class ? n_class - 1 : c);
  float v = acc + bf2f(w1m[(long)c * kNH + h]) + b1[h];
  a1[i] = v;
  h1b[i] = f2bf(v > 0.f ? v : 0.f);
  if (h < kNIn) xb[b * 16 + h] = f2bf(x[b * kNIn + h]);
}

// In place: A += bias; H = bf16(ReLU(A)).
__global__ void k_bias_relu(long n, int N, float* __restrict__ a, const float* __restrict__ bias,
                            uint16_t* __restrict__ hb) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    float v = a[i] + bias[i % N];
    a[i] = v;
    hb[i] = f2bf(v > 0.f ? v : 0.f);
  }
}

// Softmax cross-entropy over 64 logits per sample (one wave per sample, four
// per block): dZ = (softmax(z) - onehot(label)) / B, loss += (lse - z_label) / B
// (one atomic per block).
__global__ void __launch_bounds__(256) k_softmax_ce(int B, float* __restrict__ z, const float* __restrict__ b3,
                                                    const int* __restrict__ label, float* __restrict__ dz,
                                                    uint16_t* __restrict__ dzb, float* __restrict__ loss) {
  __shared__ float part[4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const long b = (long)blockIdx.x * 4 + w;
  float l = 0.f;
  if (b < B) {
    float v = z[b * kNOut + lane] + b3[lane];
    z[b * kNOut + lane] = v;
    float mx = v;
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
    float e = expf(v - mx);
    float s = e;
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    int lab = label[b];
    float g = (e / s - (lane == lab ? 1.f : 0.f)) / (float)B;
    dz[b * kNOut + lane] = g;
    dzb[b * kNOut + lane] = f2bf(g);
    l = __shfl((logf(s) - (v - mx)) / (float)B, lab);
  }
  if (lane == 0) part[w] = l;
  __syncthreads();
  if (threadIdx.x == 0 && loss) atomicAdd(loss, ((part[0] + part[1]) + part[2]) + part[3]);
}

// In place: A += bias (no activation; the logits).
__global__ void k_bias_relu_noact(long n, int N, float* __restrict__ a, const float* __restrict__ bias) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    a[i] = a[i] + bias[i % N];
}

// dA = dH * 1[A > 0]; dAb = bf16(dA).
__global__ void k_relu_grad(long n, float* __restrict__ dh, const float* __restrict__ a,
                            uint16_t* __restrict__ dab) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    float g = a[i] > 0.f ? dh[i] : 0.f;
    dh[i] = g;
    dab[i] = f2bf(g);
  }
}

// Sums over the batch are split into row slices: slice p (blockIdx.y) covers
// rows [p R, min(B, (p+1) R)) and writes its partial sums to part + p n_out;
// k_sum_parts then adds the slices in slice order, so every sum is taken in
// the same order on every run.

// Partial column sums of a [B x N] float matrix (bias gradients): 64 columns
// per block, its four waves take every fourth row, then add in wave order.
__global__ void __launch_bounds__(256) k_colsum_part(int B, int N, int R, const float* __restrict__ d,
                                                     float* __restrict__ part) {
  __shared__ float red[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int n = blockIdx.x * 64 + lane;
  const int b0 = blockIdx.y * R, b1 = min(B, b0 + R);
  float s = 0.f;
  if (n < N)
    for (int b = b0 + w; b < b1; b += 4) s += d[(long)b * N + n];
  red[w][lane] = s;
  __syncthreads();
  if (w == 0 && n < N) part[(long)blockIdx.y * N + n] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

// Partial first-layer input-weight gradients: dW1x[h][k] = sum_b
// bf16(dA1)[b][h] bf16(x)[b][k] (float accumulation); thread h owns a row of
// dW1x.  part holds [P][128 x 6].
__global__ void __launch_bounds__(kNH) k_w1x_part(int B, int R, const uint16_t* __restrict__ da1b,
                                                  const uint16_t* __restrict__ xb, float* __restrict__ part) {
  const int h = threadIdx.x;
  const int b0 = blockIdx.y * R, b1 = min(B, b0 + R);
  float s[kNIn] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int b = b0; b < b1; b++) {
    const float g = bf2f(da1b[(long)b * kNH + h]);
#pragma unroll
    for (int k = 0; k < kNIn; k++) s[k] += g * bf2f(xb[(long)b * 16 + k]);
  }
#pragma unroll
  for (int k = 0; k < kNIn; k++) part[(long)blockIdx.y * (kNH * kNIn) + h * kNIn + k] = s[k];
}

// Partial class-row gradients of the first layer: dW1m[c][h] = sum over rows
// b with cls[b] = c of dA1[b][h] (float).  Block (x, y) accumulates classes
// [16 x, 16 x + 16) over row slice y in LDS; thread h owns column h, so each
// sum runs in row order.  part holds [P][n_class x 128].
__global__ void __launch_bounds__(kNH) k_w1m_part(int B, int R, int n_class, const float* __restrict__ da1,
                                                  const int* __restrict__ cls, float* __restrict__ part) {
  __shared__ float acc[16][kNH];
  const int h = threadIdx.x;
  const int c0 = blockIdx.x * 16;
  const int b0 = blockIdx.y * R, b1 = min(B, b0 + R);
#pragma unroll
  for (int c = 0; c < 16; c++) acc[c][h] = 0.f;
  for (int b = b0; b < b1; b++) {
    int c = cls[b];
    c = (c < 0 ? 0 : (c >= n_class ? n_class - 1 : c)) - c0;
    if (c >= 0 && c < 16) acc[c][h] += da1[(long)b * kNH + h];
  }
  const int nc = min(16, n_class - c0);
  for (int c = 0; c < nc; c++) part[(long)blockIdx.y * n_class * kNH + (long)(c0 + c) * kNH + h] = acc[c][h];
}

// out[i] = sum over p = 0 .. P-1, in order, of part[p n + i].
__global__ void k_sum_parts(long n, int P, const float* __restrict__ part, float* __restrict__ out) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    float s = 0.f;
#pragma unroll 8
    for (int p = 0; p < P; p++) s += part[(long)p * n + i];
    out[i] = s;
  }
}

// Adam on the float master copy; refreshes the bf16 copy.
__global__ void k_adam(long n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, uint16_t* __restrict__ pb, float lr, float c1, float c2) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    float gi = g[i];
    float mi = b1 * m[i] + (1.f - b1) * gi;
    float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    float mh = mi / c1, vh = vi / c2;
    float w = p[i] - lr * mh / (sqrtf(vh) + eps);
    p[i] = w;
    pb[i] = f2bf(w);
  }
}

}  // namespace gnav

using namespace gnav;

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

struct gnav_mlp {
  gnav_ctx* owner = nullptr;  // the context that created it (its bindings live there)
  int n_class = 0, max_batch = 0;
  long n_params = 0;
  long o_w1x, o_w1m, o_b1, o_w2, o_b2, o_w3, o_b3;
  long step = 0;
  // parameters: float master, bf16 copy, gradients, Adam moments
  float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  uint16_t* pb = nullptr;
  // activations for max_batch samples
  float *a1 = nullptr, *a2 = nullptr, *z = nullptr, *dz = nullptr, *dh = nullptr, *loss = nullptr;
  uint16_t *xb = nullptr, *h1b = nullptr, *h2b = nullptr, *dzb = nullptr, *da2b = nullptr, *da1b = nullptr;
  float* part = nullptr;  // partial sums of split reductions (kPartFloats)
  std::vector<void*> allocs;
  ~gnav_mlp() {
    for (void* q : allocs) (void)hipFree(q);
  }
  template <class T>
  hipError_t alloc(T** ptr, size_t count) {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(count * sizeof(T), 16));
    if (e == hipSuccess) {
      allocs.push_back(q);
      *ptr = (T*)q;
      e = hipMemset(q, 0, std::max<size_t>(count * sizeof(T), 16));
    }
    return e;
  }
};

namespace gnav {
const gnav_ctx* mlp_owner(const gnav_mlp* q) { return q ? q->owner : nullptr; }

bool mlp_view(const gnav_mlp* q, MlpView* v) {
  if (!q || !v) return false;
  v->w1x = q->pb + q->o_w1x;
  v->w1m = q->pb + q->o_w1m;
  v->w2 = q->pb + q->o_w2;
  v->w3 = q->pb + q->o_w3;
  v->b1 = q->p + q->o_b1;
  v->b2 = q->p + q->o_b2;
  v->b3 = q->p + q->o_b3;
  v->n_class = q->n_class;
  return true;
}
}  // namespace gnav

namespace {

unsigned blocks_for(long n, int bs = 256) { return (unsigned)std::min<long>((n + bs - 1) / bs, 65535L * 8); }

constexpr long kPartFloats = 64L * kNH * kNH;  // 4 MB of partial sums
constexpr int kMaxSlices = 64;
constexpr int kMaxClass = 4096;
// one slice of every split reduction fits: class rows of dW1m, GEMM outputs
static_assert((long)kMaxClass * kNH <= kPartFloats && (long)kNH * kNH <= kPartFloats, "partial buffer");

// Row slices for a sum over n rows into n_out outputs: slices of at least
// `min_rows` rows, at most kMaxSlices of them, and within the partial buffer.
int slices(long n, long n_out, int min_rows, int* rows) {
  long P = (n + min_rows - 1) / min_rows;
  P = std::min<long>(P, std::min<long>(kMaxSlices, std::max<long>(1, kPartFloats / n_out)));
  P = std::max<long>(P, 1);
  long R = (n + P - 1) / P;
  *rows = (int)R;
  return (int)((n + R - 1) / R);
}

hipError_t sum_parts(long n, int P, const float* part, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_parts, dim3(blocks_for(n)), dim3(256), 0, st, n, P, part, out);
  return hipGetLastError();
}

// C = A B (see k_gemm_bf16).  Products with few output tiles and a long sum
// (the weight gradients, k = batch) split the sum into slices of at least 128
// so that enough waves run, then add the slices in order.
hipError_t gemm(gnav_mlp* q, int M, int N, int K, const uint16_t* A, long sam, long sak, const uint16_t* B,
                long sbk, long sbn, float* C, long ldc, hipStream_t st) {
  long tiles = (long)(M / 16) * (N / 16);
  unsigned gx = (unsigned)((tiles + 3) / 4);
  if (tiles < 512 && K >= 256 && ldc == N) {
    int kc = 0;
    int P = slices(K / 16, (long)M * N, 8, &kc);
    kc *= 16;
    hipLaunchKernelGGL(k_gemm_bf16, dim3(gx, (unsigned)P), dim3(256), 0, st, M, N, K, kc, A, sam, sak, B, sbk,
                       sbn, q->part, (long)N, (long)M * N);
    hipError_t e = hipGetLastError();
    return e != hipSuccess ? e : sum_parts((long)M * N, P, q->part, C, st);
  }
  hipLaunchKernelGGL(k_gemm_bf16, dim3(gx), dim3(256), 0, st, M, N, K, K, A, sam, sak, B, sbk, sbn, C, ldc, 0L);
  return hipGetLastError();
}

// Bias gradient: out[n] = sum over the Bn rows of d[b][n].
hipError_t colsum(gnav_mlp* q, int Bn, int N, const float* d, float* out, hipStream_t st) {
  int R = 0;
  int P = slices(Bn, N, 128, &R);
  hipLaunchKernelGGL(k_colsum_part, dim3((unsigned)((N + 63) / 64), (unsigned)P), dim3(256), 0, st, Bn, N, R, d,
                     q->part);
  hipError_t e = hipGetLastError();
  return e != hipSuccess ? e : sum_parts(N, P, q->part, out, st);
}

// Forward and backward for a batch; gradients land in mlp->g.
hipError_t run_grad(gnav_mlp* q, int Bn, const float* x, const int* cls, const int* label, hipStream_t st) {
  hipError_t e;
  const uint16_t* w1x = q->pb + q->o_w1x;
  const uint16_t* w1m = q->pb + q->o_w1m;
  const uint16_t* w2 = q->pb + q->o_w2;
  const uint16_t* w3 = q->pb + q->o_w3;
  if ((e = launch_zero(q->g, (size_t)((q->n_params + 1) / 2), st)) != hipSuccess) return e;
  if ((e = launch_zero(q->loss, 1, st)) != hipSuccess) return e;
  // forward
  hipLaunchKernelGGL(k_layer1, dim3(blocks_for((long)Bn * kNH)), dim3(256), 0, st, Bn, x, cls, q->n_class, w1x,
                     w1m, q->p + q->o_b1, q->xb, q->a1, q->h1b);
  if ((e = gemm(q, Bn, kNH, kNH, q->h1b, kNH, 1, w2, 1, kNH, q->a2, kNH, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_bias_relu, dim3(blocks_for((long)Bn * kNH)), dim3(256), 0, st, (long)Bn * kNH, kNH, q->a2,
                     q->p + q->o_b2, q->h2b);
  if ((e = gemm(q, Bn, kNOut, kNH, q->h2b, kNH, 1, w3, 1, kNH, q->z, kNOut, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_softmax_ce, dim3((unsigned)((Bn + 3) / 4)), dim3(256), 0, st, Bn, q->z, q->p + q->o_b3,
                     label, q->dz, q->dzb, q->loss);
  // backward
  float* g = q->g;
  // dW3 = dZb^T H2b : [64 x B] [B x 128]
  if ((e = gemm(q, kNOut, kNH, Bn, q->dzb, 1, kNOut, q->h2b, kNH, 1, g + q->o_w3, kNH, st)) != hipSuccess)
    return e;
  if ((e = colsum(q, Bn, kNOut, q->dz, g + q->o_b3, st)) != hipSuccess) return e;
  // dH2 = dZb W3 : [B x 64] [64 x 128]
  if ((e = gemm(q, Bn, kNH, kNOut, q->dzb, kNOut, 1, w3, kNH, 1, q->dh, kNH, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_relu_grad, dim3(blocks_for((long)Bn * kNH)), dim3(256), 0, st, (long)Bn * kNH, q->dh, q->a2,
                     q->da2b);
  if ((e = colsum(q, Bn, kNH, q->dh, g + q->o_b2, st)) != hipSuccess) return e;
  // dW2 = dA2b^T H1b : [128 x B] [B x 128]
  if ((e = gemm(q, kNH, kNH, Bn, q->da2b, 1, kNH, q->h1b, kNH, 1, g + q->o_w2, kNH, st)) != hipSuccess) return e;
  // dH1 = dA2b W2 : [B x 128] [128 x 128]
  if ((e = gemm(q, Bn, kNH, kNH, q->da2b, kNH, 1, w2, kNH, 1, q->dh, kNH, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_relu_grad, dim3(blocks_for((long)Bn * kNH)), dim3(256), 0, st, (long)Bn * kNH, q->dh, q->a1,
                     q->da1b);
  if ((e = colsum(q, Bn, kNH, q->dh, g + q->o_b1, st)) != hipSuccess) return e;
  // first layer: dW1x from the bf16 copies, dW1m per class row from dA1
  int R = 0;
  int P = slices(Bn, (long)kNH * kNIn, 128, &R);
  hipLaunchKernelGGL(k_w1x_part, dim3(1, (unsigned)P), dim3(kNH), 0, st, Bn, R, q->da1b, q->xb, q->part);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = sum_parts((long)kNH * kNIn, P, q->part, g + q->o_w1x, st)) != hipSuccess) return e;
  const long n_m = (long)q->n_class * kNH;
  P = slices(Bn, n_m, 128, &R);
  hipLaunchKernelGGL(k_w1m_part, dim3((unsigned)((q->n_class + 15) / 16), (unsigned)P), dim3(kNH), 0, st, Bn, R,
                     q->n_class, q->dh, cls, q->part);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return sum_parts(n_m, P, q->part, g + q->o_w1m, st);
}

}  // namespace

extern "C" {

gnav_status gnav_mlp_create(gnav_ctx* ctx, int32_t n_class, int32_t max_batch, const float* params,
                            gnav_mlp** out) {
  if (!ctx || !out || !params || n_class <= 0 || n_class > kMaxClass || max_batch <= 0 || max_batch % 16 != 0 ||
      max_batch > (1 << 22))
    return GNAV_EINVAL;
  *out = nullptr;
  gnav_mlp* q = new (std::nothrow) gnav_mlp();
  if (!q) return GNAV_ENOMEM;
  q->owner = ctx;
  q->n_class = n_class;
  q->max_batch = max_batch;
  long o = 0;
  q->o_w1x = o; o += (long)kNH * kNIn;
  q->o_w1m = o; o += (long)n_class * kNH;
  q->o_b1 = o; o += kNH;
  q->o_w2 = o; o += (long)kNH * kNH;
  q->o_b2 = o; o += kNH;
  q->o_w3 = o; o += (long)kNOut * kNH;
  q->o_b3 = o; o += kNOut;
  q->n_params = o;
  long Bn = max_batch;
  hipError_t e;
  if ((e = q->alloc(&q->p, o)) != hipSuccess || (e = q->alloc(&q->g, o + 2)) != hipSuccess ||
      (e = q->alloc(&q->m, o)) != hipSuccess || (e = q->alloc(&q->v, o)) != hipSuccess ||
      (e = q->alloc(&q->pb, o)) != hipSuccess || (e = q->alloc(&q->a1, Bn * kNH)) != hipSuccess ||
      (e = q->alloc(&q->a2, Bn * kNH)) != hipSuccess || (e = q->alloc(&q->z, Bn * kNOut)) != hipSuccess ||
      (e = q->alloc(&q->dz, Bn * kNOut)) != hipSuccess || (e = q->alloc(&q->dh, Bn * kNH)) != hipSuccess ||
      (e = q->alloc(&q->loss, 2)) != hipSuccess || (e = q->alloc(&q->xb, Bn * 16)) != hipSuccess ||
      (e = q->alloc(&q->h1b, Bn * kNH)) != hipSuccess || (e = q->alloc(&q->h2b, Bn * kNH)) != hipSuccess ||
      (e = q->alloc(&q->dzb, Bn * kNOut)) != hipSuccess || (e = q->alloc(&q->da2b, Bn * kNH)) != hipSuccess ||
      (e = q->alloc(&q->da1b, Bn * kNH)) != hipSuccess || (e = q->alloc(&q->part, kPartFloats)) != hipSuccess) {
    delete q;
    return e == hipErrorOutOfMemory ? GNAV_ENOMEM : GNAV_EHIP;
  }
  if (hipMemcpy(q->p, params, o * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
    delete q;
    return GNAV_EHIP;
  }
  hipLaunchKernelGGL(k_cast_bf16, dim3(blocks_for(o)), dim3(256), 0, 0, q->p, q->pb, o);
  if (hipDeviceSynchronize() != hipSuccess) {
    delete q;
    return GNAV_EHIP;
  }
  *out = q;
  return GNAV_OK;
}

int64_t gnav_mlp_n_params(const gnav_mlp* q) { return q ? q->n_params : -1; }

gnav_status gnav_mlp_grad(gnav_ctx* ctx, gnav_mlp* q, int64_t batch, const float* x_dev, const int32_t* cls_dev,
                          const int32_t* label_dev, float* grad_dev, float* loss_dev, void* stream) {
  if (!ctx || !q || !x_dev || !cls_dev || !label_dev) return GNAV_EINVAL;
  if (batch <= 0 || batch > q->max_batch || batch % 16 != 0) return GNAV_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  if (run_grad(q, (int)batch, x_dev, cls_dev, label_dev, st) != hipSuccess) return GNAV_EHIP;
  if (grad_dev && hipMemcpyAsync(grad_dev, q->g, q->n_params * sizeof(float), hipMemcpyDeviceToDevice, st) !=
                      hipSuccess)
    return GNAV_EHIP;
  if (loss_dev && hipMemcpyAsync(loss_dev, q->loss, sizeof(float), hipMemcpyDeviceToDevice, st) != hipSuccess)
    return GNAV_EHIP;
  return GNAV_OK;
}

gnav_status gnav_mlp_adam(gnav_ctx* ctx, gnav_mlp* q, float lr, void* stream) {
  if (!ctx || !q || !(lr > 0)) return GNAV_EINVAL;
  q->step++;
  float c1 = (float)(1.0 - std::pow(0.9, (double)q->step));
  float c2 = (float)(1.0 - std::pow(0.999, (double)q->step));
  hipLaunchKernelGGL(k_adam, dim3(blocks_for(q->n_params)), dim3(256), 0, (hipStream_t)stream, q->n_params, q->p,
                     q->g, q->m, q->v, q->pb, lr, c1, c2);
  return hipGetLastError() == hipSuccess ? GNAV_OK : GNAV_EHIP;
}

gnav_status gnav_mlp_forward(gnav_ctx* ctx, gnav_mlp* q, int64_t batch, const float* x_dev,
                             const int32_t* cls_dev, float* logits_dev, void* stream) {
  if (!ctx || !q || !x_dev || !cls_dev || !logits_dev) return GNAV_EINVAL;
  if (batch <= 0 || batch > q->max_batch || batch % 16 != 0) return GNAV_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  int Bn = (int)batch;
  hipLaunchKernelGGL(k_layer1, dim3(blocks_for((long)Bn * kNH)), dim3(256), 0, st, Bn, x_dev, cls_dev, q->n_class,
                     q->pb + q->o_w1x, q->pb + q->o_w1m, q->p + q->o_b1, q->xb, q->a1, q->h1b);
  if (gemm(q, Bn, kNH, kNH, q->h1b, kNH, 1, q->pb + q->o_w2, 1, kNH, q->a2, kNH, st) != hipSuccess)
    return GNAV_EHIP;
  hipLaunchKernelGGL(k_bias_relu, dim3(blocks_for((long)Bn * kNH)), dim3(256), 0, st, (long)Bn * kNH, kNH, q->a2,
                     q->p + q->o_b2, q->h2b);
  if (gemm(q, Bn, kNOut, kNH, q->h2b, kNH, 1, q->pb + q->o_w3, 1, kNH, logits_dev, kNOut, st) != hipSuccess)
    return GNAV_EHIP;
  hipLaunchKernelGGL(k_bias_relu_noact, dim3(blocks_for((long)Bn * kNOut)), dim3(256), 0, st, (long)Bn * kNOut,
                     kNOut, logits_dev, q->p + q->o_b3);
  return hipGetLastError() == hipSuccess ? GNAV_OK : GNAV_EHIP;
}

gnav_status gnav_mlp_score(gnav_ctx* ctx, gnav_mlp* q, int64_t n, const float* x_dev, const int32_t* cls_dev,
                           float* logits_dev, int32_t* pred_dev, void* stream) {
  if (!ctx || !q || n < 0 || (n > 0 && (!x_dev || !cls_dev))) return GNAV_EINVAL;
  if (n > (1L << 40)) return GNAV_EINVAL;
  MlpView M;
  if (!mlp_view(q, &M)) return GNAV_EINVAL;
  return launch_mlp_score(M, (long)n, x_dev, cls_dev, logits_dev, pred_dev, (hipStream_t)stream) == hipSuccess
             ? GNAV_OK
             : GNAV_EHIP;
}

gnav_status gnav_mlp_get_params(gnav_ctx* ctx, gnav_mlp* q, float* params_host) {
  if (!ctx || !q || !params_host) return GNAV_EINVAL;
  if (hipDeviceSynchronize() != hipSuccess) return GNAV_EHIP;
  if (hipMemcpy(params_host, q->p, q->n_params * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
    return GNAV_EHIP;
  return GNAV_OK;
}

gnav_status gnav_mlp_free(gnav_ctx* ctx, gnav_mlp* q) {
  if (!ctx) return GNAV_EINVAL;
  (void)hipDeviceSynchronize();
  if (q) gnav::unbind_mlp(q->owner, q);
  delete q;
  return GNAV_OK;
}

}  // extern "C"

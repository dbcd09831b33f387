// gnav_learned.h -- inference of the candidate-ordering network on bf16 MFMA,
// shared by the transport kernel and the ComputeStep query kernel.
//
// The network (two hidden layers of 128 ReLU units over 6 features and a
// one-hot of the mother's ordering class, 64 logits, one per candidate
// position of the start voxel node) predicts which daughter limits a step, so
// that daughter's exact entry distance is evaluated first and bounds the
// others.  The predicted position is the argmax of the logits (lowest
// position on ties).  The prediction only orders the search: the step found
// is the same whatever it predicts.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gnav_internal.h"

namespace gnav {

typedef short lbf16x4 __attribute__((ext_vector_type(4)));
typedef float lf32x4 __attribute__((ext_vector_type(4)));

// float -> bf16 bits, round to nearest even (quiet NaN kept).
__device__ __forceinline__ uint16_t lf2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float lbf2f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

// Four consecutive bf16 values as one MFMA operand (8-byte aligned loads).
__device__ __forceinline__ lbf16x4 load_bf16x4(const uint16_t* p) {
  return *reinterpret_cast<const lbf16x4*>(p);
}

// Scores n rows whose bf16 features are xf[i][0..5] and ordering classes
// cls[i] (both in LDS), and writes the highest-scoring candidate position of
// each row over cls[i].  Called by every thread of a block of WAVES waves.
//
// v_mfma_f32_16x16x16_bf16 (float accumulation), per lane l: A rows
// m = l % 16, k = 4 (l / 16) + 0..3; B columns n = l % 16, same k; D columns
// n = l % 16, rows 4 (l / 16) + 0..3.  Each wave takes 16 rows at a time and
// computes every layer transposed, H^T = W X^T: the weights are the A
// operand (row = output unit l % 16) and the activations the B operand
// (column = row of the batch), so the accumulator of output tile t holds,
// per lane, units 16 t + 4 (l / 16) + 0..3 of row l % 16, which is exactly
// the B operand of the next layer's k-slice t: activations stay in
// registers and never pass through LDS.
//
// Kept out of line (the MFMA operands would otherwise raise the register
// count of the calling loop); it takes the weights by value so that the
// caller's argument block is never addressed from the call.  With LOGITS the
// 64 logits of row i also go to logits[64 i + c] (float, global memory).
// A zero the compiler cannot see through (one instruction).
__device__ __forceinline__ long opaque_zero() {
  int z;
  asm volatile("v_mov_b32 %0, 0" : "=v"(z));
  return (long)z;
}

template <int WAVES, bool LOGITS = false>
__device__ __attribute__((noinline)) void learned_predict(const MlpView M, uint16_t (*xf)[6], uint16_t* cls_io,
                                                          int n, float* logits = nullptr) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r = lane & 15, q = lane >> 4;
  for (int row0 = 16 * w; row0 < n; row0 += 16 * WAVES) {
    // The weight loads of each 16-row tile are issued inside its iteration
    // and layer by layer: an opaque zero added to every weight address keeps
    // the compiler from hoisting all of them out of the loop (they would hold
    // some 130 registers at once, which an out-of-line function must save
    // and restore around every call).
    const long wz = opaque_zero();
    const int li = row0 + r;
    const bool valid = li < n;
    const int cls = valid ? cls_io[li] : 0;
    // layer 1: K = 6 inputs padded to 16; + W1m[class] + b1, ReLU
    lbf16x4 x;
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const int k = 4 * q + j;
      x[j] = (short)(k < 6 && valid ? xf[li][k] : 0);
    }
    lbf16x4 h1[8];
#pragma unroll
    for (int t = 0; t < 8; t++) {
      lbf16x4 wa;
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const int k = 4 * q + j;
        wa[j] = (short)(k < 6 ? M.w1x[wz + (16 * t + r) * 6 + k] : 0);
      }
      lf32x4 acc = {0.f, 0.f, 0.f, 0.f};
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wa, x, acc, 0, 0, 0);
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const int u = 16 * t + 4 * q + j;
        const float v = acc[j] + lbf2f(M.w1m[(long)cls * 128 + u]) + M.b1[u];
        h1[t][j] = (short)lf2bf(v > 0.f ? v : 0.f);
      }
    }
    // layer 2 + b2, ReLU (each tile's eight A operands loaded before its MFMA chain)
    lbf16x4 h2[8];
#pragma unroll
    for (int t = 0; t < 8; t++) {
      lbf16x4 wa[8];
#pragma unroll
      for (int kt = 0; kt < 8; kt++) wa[kt] = load_bf16x4(M.w2 + wz + (16 * t + r) * 128 + 16 * kt + 4 * q);
      lf32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kt = 0; kt < 8; kt++) acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wa[kt], h1[kt], acc, 0, 0, 0);
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const float v = acc[j] + M.b2[16 * t + 4 * q + j];
        h2[t][j] = (short)lf2bf(v > 0.f ? v : 0.f);
      }
    }
    // layer 3 + b3: 64 logits; this lane holds candidates 16 t + 4 q + j
    float best_v = 0.f;
    int best_c = -1;
#pragma unroll
    for (int t = 0; t < 4; t++) {
      lbf16x4 wa[8];
#pragma unroll
      for (int kt = 0; kt < 8; kt++) wa[kt] = load_bf16x4(M.w3 + wz + (16 * t + r) * 128 + 16 * kt + 4 * q);
      lf32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kt = 0; kt < 8; kt++) acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wa[kt], h2[kt], acc, 0, 0, 0);
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const int c = 16 * t + 4 * q + j;
        const float v = acc[j] + M.b3[c];
        if (LOGITS && valid) logits[(long)li * 64 + c] = v;
        if (best_c < 0 || v > best_v) {  // candidates arrive in increasing order
          best_v = v;
          best_c = c;
        }
      }
    }
    // highest logit over the four lanes of the row; the lowest position on ties
#pragma unroll
    for (int off = 16; off <= 32; off <<= 1) {
      const float ov = __shfl_xor(best_v, off);
      const int oc = __shfl_xor(best_c, off);
      if (ov > best_v || (ov == best_v && oc < best_c)) {
        best_v = ov;
        best_c = oc;
      }
    }
    if (q == 0 && valid) cls_io[li] = (uint16_t)best_c;
  }
}

// Features of a step in mother LV record L at mother-frame point pl and
// direction vl: the point relative to the voxel grid's centre over its half
// size, then the direction, rounded to bf16; and the ordering class clamped
// to the network's range.
__device__ __forceinline__ void learned_features(const LRec& L, V3 pl, V3 vl, int n_class, uint16_t* xf,
                                                 uint16_t* cls) {
  const double pc[3] = {pl.x, pl.y, pl.z};
#pragma unroll
  for (int ax = 0; ax < 3; ax++) {
    const double half = 0.5 * L.n[ax] * L.vw[ax];
    xf[ax] = lf2bf((float)((pc[ax] - (L.vlo[ax] + half)) / half));
  }
  xf[3] = lf2bf((float)vl.x);
  xf[4] = lf2bf((float)vl.y);
  xf[5] = lf2bf((float)vl.z);
  const int c = L.lclass;
  *cls = (uint16_t)(c < 0 ? 0 : (c >= n_class ? n_class - 1 : c));
}

}  // namespace gnav

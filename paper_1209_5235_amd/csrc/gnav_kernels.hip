// gnav_kernels.hip -- navigation query kernels (locate, ComputeStep,
// ComputeSafety), the free path of Alg. 1 alone, small reset kernels, and
// the dispatch of the transport kernel to the build for the chosen pool size.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "gnav_device.h"
#include "gnav_internal.h"
#include "gnav_learned.h"
#include "gnav_physics.h"

namespace gnav {

// ---------------------------------------------------------------------------
// Query kernels (one thread per query)
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256) k_locate(DevGeom G, int W, int tbase, long n, const double* pos,
                                                const double* dir, int* out) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  NavCount<false> nc;
  V3 p{pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
  V3 v{0, 0, 0};
  bool hv = dir != nullptr;
  if (hv) v = V3{dir[3 * i], dir[3 * i + 1], dir[3 * i + 2]};
  int T = locate(G, W, p, hv, v, nc);
  out[i] = T < 0 ? -1 : T - tbase;
}

// Exit normal at the end point q (global) of a step from touchable T that
// ended on the boundary of the mother (lim < 0) or of daughter slot lim: the
// outward normal of the mother, or the inward normal of the entered daughter,
// rotated to the global frame (the world->local maps are rotations, so a
// direction returns through the transposed matrix).
__device__ __forceinline__ int exit_normal(const DevGeom& G, int T, const TRec& tr, int lim, V3 q, V3& ng) {
  const int S = lim >= 0 ? tr.child_base + lim : T;
  const TRec ts = lim >= 0 ? G.t[S] : tr;
  const LRec& L = G.lv[ts.lv];
  V3 ql, dummy;
  touchable_frame(G, S, trec_kind(ts), q, V3{0.0, 0.0, 1.0}, ql, dummy);
  V3 nl;
  const int faces = solid_normal(L.info, L.par, ql, nl);
  if (lim >= 0) nl = V3{-nl.x, -nl.y, -nl.z};
  if (trec_kind(ts) == 0) {
    ng = nl;
  } else {
    const double* m = G.t_xf + (size_t)S * 12;
    ng = V3{m[0] * nl.x + m[3] * nl.y + m[6] * nl.z, m[1] * nl.x + m[4] * nl.y + m[7] * nl.z,
            m[2] * nl.x + m[5] * nl.y + m[8] * nl.z};
  }
  return faces > 1 ? GNAV_NORMAL_EDGE : GNAV_NORMAL_FACE;
}

// ComputeStep queries, one per thread (256 per block).  With the learned
// order every thread first gathers its features into LDS and the block
// scores all of them on MFMA (rows of threads without a voxelised mother
// are scored too and ignored), so no thread may leave before that.
template <int PREC, int ORDER>
__global__ void __launch_bounds__(256) k_step(StepArgs a) {
  const DevGeom& G = a.G;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const bool act = i < a.n;
  NavCount<false> nc;
  V3 p{0.0, 0.0, 0.0}, v{0.0, 0.0, 1.0};
  int T = -1;
  if (act) {
    p = V3{a.pos[3 * i], a.pos[3 * i + 1], a.pos[3 * i + 2]};
    v = V3{a.dir[3 * i], a.dir[3 * i + 1], a.dir[3 * i + 2]};
    if (a.touch) T = (a.touch[i] < 0 || a.touch[i] >= a.tcount) ? -1 : a.touch[i] + a.tbase;
    else T = locate(G, a.W, p, true, v, nc);
  }
  TRec tr{0, -1, 0, 0};
  V3 pl{0.0, 0.0, 0.0}, vl{0.0, 0.0, 1.0};
  if (T >= 0) {
    tr = G.t[T];
    touchable_frame(G, T, trec_kind(tr), p, v, pl, vl);
  }
  int pred = -1;
  if constexpr (ORDER == kOrderLearned) {
    __shared__ uint16_t xf[256][6];
    __shared__ uint16_t cls[256];
    const int t = threadIdx.x;
    bool elig = false;
    if (T >= 0) {
      const LRec& L = G.lv[tr.lv];
      elig = L.lclass >= 0 && L.wide && L.dau_cnt > 0;
    }
    if (elig) {
      learned_features(G.lv[tr.lv], pl, vl, a.mlp.n_class, xf[t], &cls[t]);
    } else {
#pragma unroll
      for (int k = 0; k < 6; k++) xf[t][k] = 0;
      cls[t] = 0;
    }
    if (__syncthreads_or(elig)) {
      learned_predict<4>(a.mlp, xf, cls, 256);
      __syncthreads();
      if (elig) pred = cls[t];
    }
  }
  if (!act) return;
  if (T < 0) {
    a.step[i] = kInf;
    a.lim[i] = kLimMother;
    if (a.next) a.next[i] = -1;
    if (a.saf) a.saf[i] = 0.0;
    if (a.normal) a.normal[3 * i] = a.normal[3 * i + 1] = a.normal[3 * i + 2] = 0.0;
    if (a.normal_valid) a.normal_valid[i] = GNAV_NORMAL_NONE;
    return;
  }
  int lim;
  double saf;
  double s = compute_step_p<false, ORDER, PREC>(G, G.lv[tr.lv], tr.lv, pl, vl, lim, saf, nc, pred, nullptr);
  if (a.max_step) {
    double ms = a.max_step[i];
    if (ms < 0.0) ms = 0.0;
    if (ms <= s) {  // false for NaN: no limit
      s = ms;
      lim = kLimMaxStep;
    }
  }
  a.step[i] = s;
  a.lim[i] = lim;
  if (a.saf) a.saf[i] = saf;
  const bool crossed = lim != kLimMaxStep && s < kInf;
  const V3 q{p.x + s * v.x, p.y + s * v.y, p.z + s * v.z};
  if (a.next) {
    int nt = T;
    if (lim != kLimMaxStep) nt = crossed ? relocate(G, T, tr, q, v, lim, nc) : -1;
    a.next[i] = nt < 0 ? -1 : nt - a.tbase;
  }
  if (a.normal || a.normal_valid) {
    V3 ng{0.0, 0.0, 0.0};
    const int code = crossed ? exit_normal(G, T, tr, lim, q, ng) : GNAV_NORMAL_NONE;
    if (a.normal) {
      a.normal[3 * i] = ng.x;
      a.normal[3 * i + 1] = ng.y;
      a.normal[3 * i + 2] = ng.z;
    }
    if (a.normal_valid) a.normal_valid[i] = code;
  }
}

template <int PREC>
__global__ void __launch_bounds__(256) k_safety(DevGeom G, int W, int tbase, int tcount, long n,
                                                const double* pos, const int* touch, double* out) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  NavCount<false> nc;
  V3 p{pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
  V3 z{0, 0, 0};
  int T = touch ? ((touch[i] < 0 || touch[i] >= tcount) ? -1 : touch[i] + tbase)
                : locate(G, W, p, false, z, nc);
  if (T < 0) {
    out[i] = 0.0;
    return;
  }
  TRec tr = G.t[T];
  V3 pl, vl;
  touchable_frame(G, T, trec_kind(tr), p, V3{0, 0, 1}, pl, vl);
  int lim;
  double saf;
  // the safety comes from the start node of a step walk along any direction
  compute_step_p<false, kOrderPlain, PREC>(G, G.lv[tr.lv], tr.lv, pl, vl, lim, saf, nc, -1, nullptr);
  out[i] = saf;
}

// Free path of Alg. 1 alone (the paper's timed phase, Alg. 2 phase 5): from
// the start point, cross boundaries accumulating the optical depth S_j = sum
// mu_i s_i (Eq. 6) until it reaches the particle's lifetime Y; the first
// interaction lies at T = t_{j-1} + (Y - S_{j-1}) / mu_j (Eq. 7).  mu is the
// paper's rho mu_Al (Eq. 9) when mu_mass > 0, else the tabulated total
// attenuation at energy E.  T = +inf when the particle leaves the world.
__global__ void __launch_bounds__(256) k_free_path(DevGeom G, int W, long n, const double* pos, const double* dir,
                                                   const double* life, double E, double mu_mass, double* t_out,
                                                   int* nb_out) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  NavCount<false> nc;
  V3 x{pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
  V3 v{dir[3 * i], dir[3 * i + 1], dir[3 * i + 2]};
  const double Y = life[i];
  int T = locate(G, W, x, true, v, nc);
  double t_prev = 0.0, S_prev = 0.0, result = kInf;
  int nb = 0;
  int imu = 0;
  double wmu = 0.0;
  if (mu_mass <= 0.0) mu_index(G, E, imu, wmu);
  while (T >= 0) {
    const TRec tr = G.t[T];
    const LRec& L = G.lv[tr.lv];
    double mu;
    if (mu_mass > 0.0) {
      mu = G.mat_rho[L.mat] * mu_mass * 0.1;
    } else {
      double pe, co, pp;
      mu_parts(G, L.mat, imu, wmu, E, pe, co, pp);
      mu = pe + co + pp;
    }
    V3 pl, vl;
    touchable_frame(G, T, trec_kind(tr), x, v, pl, vl);
    int lim;
    double saf;
    const double s = compute_step(G, L, pl, vl, lim, saf, nc);
    const double S = mu > 0 ? S_prev + s * mu : S_prev;
    if (mu > 0 && S >= Y) {
      result = t_prev + (Y - S_prev) / mu;
      break;
    }
    x = V3{x.x + s * v.x, x.y + s * v.y, x.z + s * v.z};
    t_prev = t_prev + s;
    S_prev = S;
    T = relocate(G, T, tr, x, v, lim, nc);
    nb++;
    if (nb > 1000000) break;
  }
  t_out[i] = result;
  if (nb_out) nb_out[i] = nb;
}

// The work queue's counter and, when a claim order is built, its class
// counts and cursors, zeroed in one launch (a kernel rather than a memset
// node, so the launch sequence can be captured in a graph).
__global__ void k_reset_launch(unsigned long long* queue, unsigned* claim_cnt, int claim_words) {
  if (threadIdx.x == 0) queue[0] = 0ull;
  if (claim_cnt)
    for (int i = threadIdx.x; i < claim_words; i += blockDim.x) claim_cnt[i] = 0u;
}

__global__ void k_zero_words(unsigned long long* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

// ---------------------------------------------------------------------------
// Launch wrappers
// ---------------------------------------------------------------------------

static inline unsigned grid_for(long n, int block) { return (unsigned)((n + block - 1) / block); }
hipError_t launch_locate(const DevGeom& G, int W, int tbase, long n, const double* pos,
                         const double* dir, int* out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_locate, dim3(grid_for(n, 256)), dim3(256), 0, st, G, W, tbase, n, pos, dir, out);
  return hipGetLastError();
}

hipError_t launch_step(const StepArgs& a, int prec, int order, hipStream_t st) {
  if (a.n <= 0) return hipSuccess;
  dim3 grid(grid_for(a.n, 256)), block(256);
  if (prec == kPrecScreened) hipLaunchKernelGGL((k_step<kPrecScreened, kOrderPlain>), grid, block, 0, st, a);
  else if (prec == kPrecPure) hipLaunchKernelGGL((k_step<kPrecPure, kOrderPlain>), grid, block, 0, st, a);
  else if (order == kOrderBound) hipLaunchKernelGGL((k_step<kPrecFP64, kOrderBound>), grid, block, 0, st, a);
  else if (order == kOrderLearned) hipLaunchKernelGGL((k_step<kPrecFP64, kOrderLearned>), grid, block, 0, st, a);
  else hipLaunchKernelGGL((k_step<kPrecFP64, kOrderPlain>), grid, block, 0, st, a);
  return hipGetLastError();
}

hipError_t launch_safety(const DevGeom& G, int W, int tbase, int tcount, long n, const double* pos,
                         const int* touch, double* out, int prec, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  dim3 grid(grid_for(n, 256)), block(256);
  if (prec == kPrecScreened)
    hipLaunchKernelGGL(k_safety<kPrecScreened>, grid, block, 0, st, G, W, tbase, tcount, n, pos, touch, out);
  else if (prec == kPrecPure)
    hipLaunchKernelGGL(k_safety<kPrecPure>, grid, block, 0, st, G, W, tbase, tcount, n, pos, touch, out);
  else
    hipLaunchKernelGGL(k_safety<kPrecFP64>, grid, block, 0, st, G, W, tbase, tcount, n, pos, touch, out);
  return hipGetLastError();
}

hipError_t launch_free_path(const DevGeom& G, int W, long n, const double* pos, const double* dir,
                            const double* life, double E, double mu_mass, double* t_out, int* nb_out,
                            hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_free_path, dim3(grid_for(n, 256)), dim3(256), 0, st, G, W, n, pos, dir, life, E, mu_mass,
                     t_out, nb_out);
  return hipGetLastError();
}

// The transport's candidate-ordering network on n rows of features (float
// [n][6], rounded to bf16 as the transport rounds its features) and classes:
// logits [n][64] (optional) and the predicted candidate position [n]
// (optional), 256 rows per block.
__global__ void __launch_bounds__(256) k_mlp_score(MlpView M, long n, const float* x, const int* cls,
                                                   float* logits, int* pred) {
  __shared__ uint16_t xf[256][6];
  __shared__ uint16_t cl[256];
  const int t = threadIdx.x;
  const long row0 = (long)blockIdx.x * 256;
  const long i = row0 + t;
  if (i < n) {
#pragma unroll
    for (int k = 0; k < 6; k++) xf[t][k] = lf2bf(x[6 * i + k]);
    const int c = cls[i];
    cl[t] = (uint16_t)(c < 0 ? 0 : (c >= M.n_class ? M.n_class - 1 : c));
  } else {
#pragma unroll
    for (int k = 0; k < 6; k++) xf[t][k] = 0;
    cl[t] = 0;
  }
  __syncthreads();
  const int rows = (int)std::min<long>(256, n - row0);
  if (logits) learned_predict<4, true>(M, xf, cl, rows, logits + row0 * 64);
  else learned_predict<4>(M, xf, cl, rows);
  __syncthreads();
  if (pred && i < n) pred[i] = cl[t];
}

hipError_t launch_mlp_score(const MlpView& M, long n, const float* x, const int* cls, float* logits, int* pred,
                            hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_score, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, M, n, x, cls, logits,
                     pred);
  return hipGetLastError();
}

__global__ void k_zero_words4(unsigned long long* p0, size_t n0, unsigned long long* p1, size_t n1,
                              unsigned long long* p2, size_t n2, unsigned long long* p3, size_t n3) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (size_t i = t; i < n0; i += stride) p0[i] = 0ull;
  for (size_t i = t; i < n1; i += stride) p1[i] = 0ull;
  for (size_t i = t; i < n2; i += stride) p2[i] = 0ull;
  for (size_t i = t; i < n3; i += stride) p3[i] = 0ull;
}

hipError_t launch_zero4(void* const p[4], const size_t words[4], hipStream_t st) {
  size_t n[4], most = 0;
  for (int k = 0; k < 4; k++) {
    n[k] = p[k] ? words[k] : 0;
    most = std::max(most, n[k]);
  }
  if (most == 0) return hipSuccess;
  unsigned blocks = (unsigned)std::min<size_t>((most + 255) / 256, 4096);
  hipLaunchKernelGGL(k_zero_words4, dim3(blocks), dim3(256), 0, st, (unsigned long long*)p[0], n[0],
                     (unsigned long long*)p[1], n[1], (unsigned long long*)p[2], n[2], (unsigned long long*)p[3],
                     n[3]);
  return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t words, hipStream_t st) {
  if (words == 0) return hipSuccess;
  unsigned blocks = (unsigned)std::min<size_t>((words + 255) / 256, 4096);
  hipLaunchKernelGGL(k_zero_words, dim3(blocks), dim3(256), 0, st, (unsigned long long*)p, words);
  return hipGetLastError();
}

// Energy class of a primary for the claim order: 0 for the highest energies.
// Half octaves from 1 keV (class 63 holds everything at or below 1 keV, and
// energies that are not positive finite numbers, which the transport rejects).
__device__ __forceinline__ int claim_class(double E) {
  if (!(E > 1e-3) || !(E < 1e300)) return kClaimClasses - 1;
  const int h = (int)(2.0 * log2(E * 1e3));
  return kClaimClasses - 1 - min(h, kClaimClasses - 1);
}

// What the claim kernels read of a batch.
struct ClaimArgs {
  const double* pos;
  const double* dir;
  const double* E;
  const int* event;
  const int* prim_id;
  const int* event_geom;  // null: one geometry
  long n;
  int n_events, n_geoms;
  int n_keys;             // kClaimClasses, times the geometries when event_geom is given
  unsigned* cnt;          // [n_keys] counts, then [n_keys] cursors
  ClaimRec* claim;
};

// Sort key of primary i: its energy class, preceded by its event's geometry
// when the batch spans several (the tracks of one geometry stay together, each
// geometry's highest energies first).  Keys of events or geometries out of
// range are those of geometry 0 (the transport rejects such primaries).
__device__ __forceinline__ int claim_key(const ClaimArgs& a, long i) {
  int k = claim_class(a.E[i]);
  if (a.event_geom) {
    const int ev = a.event[i];
    int g = (ev >= 0 && ev < a.n_events) ? a.event_geom[ev] : 0;
    if (g < 0 || g >= a.n_geoms) g = 0;
    k += kClaimClasses * g;
  }
  return k;
}

// Key counts of the batch (cnt[0..n_keys), zeroed before).
__global__ void __launch_bounds__(256) k_claim_count(ClaimArgs a) {
  __shared__ unsigned h[kClaimMaxKeys];
  for (int c = threadIdx.x; c < a.n_keys; c += 256) h[c] = 0;
  __syncthreads();
  for (long i = blockIdx.x * 256L + threadIdx.x; i < a.n; i += (long)gridDim.x * 256)
    atomicAdd(&h[claim_key(a, i)], 1u);
  __syncthreads();
  for (int c = threadIdx.x; c < a.n_keys; c += 256)
    if (h[c]) atomicAdd(&a.cnt[c], h[c]);
}

// Queue positions: the primaries of key c fill [start_c, start_c + cnt_c)
// in the order their blocks reserve a range (cnt[n_keys + c] is the key's
// cursor, zeroed before); the order within a key is not fixed.  Each primary
// is copied to its position (reads in the caller's order, one 72-byte record
// written per primary).
__global__ void __launch_bounds__(256) k_claim_place(ClaimArgs a) {
  __shared__ unsigned start[kClaimMaxKeys], h[kClaimMaxKeys], base[kClaimMaxKeys];
  for (int c = threadIdx.x; c < a.n_keys; c += 256) start[c] = a.cnt[c];
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned acc = 0;
    for (int c = 0; c < a.n_keys; c++) {
      const unsigned k = start[c];
      start[c] = acc;
      acc += k;
    }
  }
  // kClaimSpan primaries per thread and pass: one reservation per key and
  // pass for 256 * kClaimSpan primaries keeps the shared cursors uncontended
  constexpr int kClaimSpan = 4;
  for (long i0 = blockIdx.x * (256L * kClaimSpan); i0 < a.n; i0 += (long)gridDim.x * 256 * kClaimSpan) {
    for (int c = threadIdx.x; c < a.n_keys; c += 256) h[c] = 0;
    __syncthreads();
    int c[kClaimSpan];
    unsigned r[kClaimSpan];
#pragma unroll
    for (int k = 0; k < kClaimSpan; k++) {
      const long i = i0 + k * 256 + threadIdx.x;
      c[k] = i < a.n ? claim_key(a, i) : -1;
      r[k] = c[k] >= 0 ? atomicAdd(&h[c[k]], 1u) : 0u;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < a.n_keys; q += 256)
      if (h[q]) base[q] = start[q] + atomicAdd(&a.cnt[a.n_keys + q], h[q]);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kClaimSpan; k++) {
      if (c[k] < 0) continue;
      const long i = i0 + k * 256 + threadIdx.x;
      ClaimRec q;
#pragma unroll
      for (int j = 0; j < 3; j++) {
        q.pos[j] = a.pos[3 * i + j];
        q.dir[j] = a.dir[3 * i + j];
      }
      q.energy = a.E[i];
      q.event = a.event[i];
      q.prim_id = a.prim_id[i];
      q.index = (int)i;
      q.pad = 0;
      a.claim[base[c[k]] + r[k]] = q;
    }
    __syncthreads();
  }
}

hipError_t launch_transport(const TransportLaunch& L, hipStream_t st) {
  hipLaunchKernelGGL(k_reset_launch, dim3(1), dim3(256), 0, st, L.queue, L.n > 0 ? L.claim_cnt : nullptr,
                     2 * L.claim_keys);
  if (L.n <= 0) return hipGetLastError();
  if (L.claim) {
    // claim order: primaries by decreasing energy (per geometry), so that the
    // tracks still running when the queue runs dry are short ones
    ClaimArgs ca{L.pos, L.dir, L.energy, L.event, L.prim_id, L.event_geom, L.n, L.n_events, L.n_geoms,
                 L.claim_keys, L.claim_cnt, L.claim};
    // (few blocks for the counts: each adds its histogram to the same counters)
    const unsigned count_blocks = (unsigned)std::min<long>((L.n + 255) / 256, 256);
    hipLaunchKernelGGL(k_claim_count, dim3(count_blocks), dim3(256), 0, st, ca);
    const unsigned place_blocks = (unsigned)std::min<long>((L.n + 1023) / 1024, 1024);
    hipLaunchKernelGGL(k_claim_place, dim3(place_blocks), dim3(256), 0, st, ca);
  }
  if (L.spheres) {
    if (L.block == 64) return launch_transport_pool64_spheres(L, st);
    if (L.block == 128) return launch_transport_pool128_spheres(L, st);
    return launch_transport_pool256_spheres(L, st);
  }
  if (L.block == 64) return L.axis_boxes ? launch_transport_pool64_axis_boxes(L, st) : launch_transport_pool64(L, st);
  if (L.block == 128) return launch_transport_pool128(L, st);
  return launch_transport_pool256(L, st);
}

}  // namespace gnav

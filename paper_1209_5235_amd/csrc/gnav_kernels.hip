// gnav_kernels.hip -- navigation query kernels (locate, ComputeStep,
// ComputeSafety), the free path of Alg. 1 alone, small reset kernels, and
// the dispatch of the transport kernel to the build for the chosen pool size.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "gnav_device.h"
#include "gnav_internal.h"
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

template <int PREC>
__global__ void __launch_bounds__(256) k_step(DevGeom G, int W, int tbase, int tcount, long n,
                                              const double* pos, const double* dir, const int* touch,
                                              double* step, int* lim_out, int* next, double* saf_out) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  NavCount<false> nc;
  V3 p{pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
  V3 v{dir[3 * i], dir[3 * i + 1], dir[3 * i + 2]};
  int T = touch ? ((touch[i] < 0 || touch[i] >= tcount) ? -1 : touch[i] + tbase)
                : locate(G, W, p, true, v, nc);
  if (T < 0) {
    step[i] = kInf;
    lim_out[i] = kLimMother;
    if (next) next[i] = -1;
    if (saf_out) saf_out[i] = 0.0;
    return;
  }
  TRec tr = G.t[T];
  V3 pl, vl;
  touchable_frame(G, T, trec_kind(tr), p, v, pl, vl);
  int lim;
  double saf;
  double s = compute_step_p<false, kOrderPlain, PREC>(G, G.lv[tr.lv], tr.lv, pl, vl, lim, saf, nc, -1,
                                                      nullptr);
  step[i] = s;
  lim_out[i] = lim;
  if (saf_out) saf_out[i] = saf;
  if (next) {
    int nt = -1;
    if (s < kInf) {
      V3 q{p.x + s * v.x, p.y + s * v.y, p.z + s * v.z};
      nt = relocate(G, T, tr, q, v, lim, nc);
    }
    next[i] = nt < 0 ? -1 : nt - tbase;
  }
}

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
  compute_step(G, G.lv[tr.lv], pl, vl, lim, saf, nc);
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

// Zero a small device array (a kernel rather than a memset node, so the
// launch sequence can be captured in a graph).
__global__ void k_reset_u64(unsigned long long* p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0ull;
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

hipError_t launch_step(const DevGeom& G, int W, int tbase, int tcount, long n, const double* pos,
                       const double* dir, const int* touch, double* step, int* lim, int* next, double* saf,
                       int prec, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  dim3 grid(grid_for(n, 256)), block(256);
  if (prec == kPrecScreened)
    hipLaunchKernelGGL(k_step<kPrecScreened>, grid, block, 0, st, G, W, tbase, tcount, n, pos, dir, touch,
                       step, lim, next, saf);
  else if (prec == kPrecPure)
    hipLaunchKernelGGL(k_step<kPrecPure>, grid, block, 0, st, G, W, tbase, tcount, n, pos, dir, touch, step,
                       lim, next, saf);
  else
    hipLaunchKernelGGL(k_step<kPrecFP64>, grid, block, 0, st, G, W, tbase, tcount, n, pos, dir, touch, step,
                       lim, next, saf);
  return hipGetLastError();
}

hipError_t launch_safety(const DevGeom& G, int W, int tbase, int tcount, long n, const double* pos,
                         const int* touch, double* out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_safety, dim3(grid_for(n, 256)), dim3(256), 0, st, G, W, tbase, tcount, n, pos, touch,
                     out);
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

hipError_t launch_zero(void* p, size_t words, hipStream_t st) {
  if (words == 0) return hipSuccess;
  unsigned blocks = (unsigned)std::min<size_t>((words + 255) / 256, 4096);
  hipLaunchKernelGGL(k_zero_words, dim3(blocks), dim3(256), 0, st, (unsigned long long*)p, words);
  return hipGetLastError();
}

hipError_t launch_transport(const TransportLaunch& L, hipStream_t st) {
  hipLaunchKernelGGL(k_reset_u64, dim3(1), dim3(64), 0, st, L.queue, 1);
  if (L.n <= 0) return hipGetLastError();
  if (L.block == 64) return L.axis_boxes ? launch_transport_pool64_axis_boxes(L, st) : launch_transport_pool64(L, st);
  if (L.block == 128) return launch_transport_pool128(L, st);
  return launch_transport_pool256(L, st);
}

}  // namespace gnav

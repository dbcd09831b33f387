// gnav_kernels.hip -- navigation query kernels and the persistent gamma
// transport kernel for gfx950 (wave64).
//
// Transport follows Sec. 3.1: each photon draws an Exp(1) optical depth
// (Alg. 1, steps 1-2), spends it boundary to boundary (S_j update, Eq. 6)
// and interacts where it runs out (T = t_{j-1} + (Y - S_{j-1}) / mu_j,
// Eq. 7); after a Compton scatter a new depth is drawn.  One lane holds one
// track in registers; when a lane's track ends the wave refills its idle
// lanes together from a device work queue with one atomic per wave
// (ballot + prefix count), so no lane waits for the slowest track of its
// original batch (the load-balancing idea of Sec. 5, done in registers).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "gnav_device.h"
#include "gnav_internal.h"

namespace gnav {

// ---------------------------------------------------------------------------
// Query kernels (one thread per query)
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256) k_locate(DevGeom G, int W, int tbase, long n, const double* pos,
                                                const double* dir, int* out) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  NavCount nc{};
  V3 p{pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
  V3 v{0, 0, 0};
  bool hv = dir != nullptr;
  if (hv) v = V3{dir[3 * i], dir[3 * i + 1], dir[3 * i + 2]};
  int T = locate(G, W, p, hv, v, nc);
  out[i] = T < 0 ? -1 : T - tbase;
}

__global__ void __launch_bounds__(256) k_step(DevGeom G, int W, int tbase, int tcount, long n, const double* pos,
                                              const double* dir, const int* touch, double* step,
                                              int* lim_out, int* next) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  NavCount nc{};
  V3 p{pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
  V3 v{dir[3 * i], dir[3 * i + 1], dir[3 * i + 2]};
  int T = touch ? ((touch[i] < 0 || touch[i] >= tcount) ? -1 : touch[i] + tbase)
                : locate(G, W, p, true, v, nc);
  if (T < 0) {
    step[i] = kInf;
    lim_out[i] = kLimMother;
    if (next) next[i] = -1;
    return;
  }
  V3 pl, vl;
  touchable_frame(G, T, p, v, pl, vl);
  int lim;
  double saf;
  double s = compute_step(G, G.t_lv[T], pl, vl, lim, saf, nc);
  step[i] = s;
  lim_out[i] = lim;
  if (next) {
    int nt = -1;
    if (s < kInf) {
      V3 q{p.x + s * v.x, p.y + s * v.y, p.z + s * v.z};
      nt = relocate(G, T, q, v, lim, nc);
    }
    next[i] = nt < 0 ? -1 : nt - tbase;
  }
}

__global__ void __launch_bounds__(256) k_safety(DevGeom G, int W, int tbase, int tcount, long n, const double* pos,
                                                const int* touch, double* out) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  NavCount nc{};
  V3 p{pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
  V3 z{0, 0, 0};
  int T = touch ? ((touch[i] < 0 || touch[i] >= tcount) ? -1 : touch[i] + tbase)
                : locate(G, W, p, false, z, nc);
  if (T < 0) {
    out[i] = 0.0;
    return;
  }
  V3 pl, vl;
  touchable_frame(G, T, p, V3{0, 0, 1}, pl, vl);
  int lim;
  double saf;
  // the safety comes from the start node of a step walk along any direction
  compute_step(G, G.t_lv[T], pl, vl, lim, saf, nc);
  out[i] = saf;
}

// ---------------------------------------------------------------------------
// Transport
// ---------------------------------------------------------------------------

__device__ __forceinline__ void mu_lookup(const DevGeom& G, int mat, double E, double& pe, double& co,
                                          double& pp) {
  double x = (log(E) - G.lnE0) / G.dlnE;
  int i;
  if (x < 0) i = 0;
  else if (x >= 255.0) i = 255;
  else i = (int)x;
  double w = x - (double)i;
  w = dmin(dmax(w, 0.0), 1.0);
  const double* t = G.xs + (size_t)mat * 3 * kNNode;
  pe = (1.0 - w) * t[i] + w * t[i + 1];
  co = (1.0 - w) * t[kNNode + i] + w * t[kNNode + i + 1];
  pp = (1.0 - w) * t[2 * kNNode + i] + w * t[2 * kNNode + i + 1];
  if (E < 2.0 * kMe) pp = 0.0;
}

// Butcher-Messel sampling of the Klein-Nishina energy fraction eps = E'/E:
// a two-branch mixture (weights ln(1+2k) and (1-eps0^2)/2) with acceptance
// 1 - eps sin^2(theta) / (1 + eps^2); three draws per trial.
__device__ __forceinline__ void compton_sample(double E, Philox& rs, double& eps, double& onecost,
                                               double& sint2) {
  double k = E / kMe;
  double eps0 = 1.0 / (1.0 + 2.0 * k);
  double eps0sq = eps0 * eps0;
  double a1 = log(1.0 + 2.0 * k);
  double a2 = 0.5 * (1.0 - eps0sq);
  for (int trial = 0; trial < kMaxComptonTrials; trial++) {
    double r1 = rng_next(rs), r2 = rng_next(rs), r3 = rng_next(rs);
    double epssq;
    if (r1 * (a1 + a2) < a1) {
      eps = exp(-a1 * r2);
      epssq = eps * eps;
    } else {
      epssq = eps0sq + (1.0 - eps0sq) * r2;
      eps = sqrt(epssq);
    }
    onecost = (1.0 - eps) / (eps * k);
    sint2 = onecost * (2.0 - onecost);
    double g = 1.0 - eps * sint2 / (1.0 + epssq);
    if (r3 <= g) break;
  }
}

__device__ __forceinline__ void rotate_dir(V3& v, double cost, double sint, double phi) {
  double cp = cos(phi), sp = sin(phi);
  double a = v.x, b = v.y, c = v.z;
  double rp = sqrt(a * a + b * b);
  double nx, ny, nz;
  if (rp < 1e-12) {
    nx = sint * cp;
    ny = sint * sp;
    nz = (c >= 0 ? 1.0 : -1.0) * cost;
  } else {
    double e1x = a * c / rp, e1y = b * c / rp, e1z = -(a * a + b * b) / rp;
    double e2x = -b / rp, e2y = a / rp, e2z = 0.0;
    nx = cost * a + sint * (cp * e1x + sp * e2x);
    ny = cost * b + sint * (cp * e1y + sp * e2y);
    nz = cost * c + sint * (cp * e1z + sp * e2z);
  }
  double nn = sqrt(nx * nx + ny * ny + nz * nz);
  v = V3{nx / nn, ny / nn, nz / nn};
}

struct TransportArgs {
  DevGeom G;
  long n;
  const int* event;
  const int* prim_id;
  const double* pos;
  const double* dir;
  const double* energy;
  const int* event_geom;   // may be null
  int geom_default;
  const int* geom_tbase;   // [geoms] first touchable (global)
  int n_geoms;
  int n_events;
  uint64_t seed;
  double ecut;
  long max_steps;
  double* edep_t;
  double* edep_ev;
  double* esc_ev;
  unsigned long long* counters;
  unsigned long long* queue;  // [0]: next primary
  gnav_logrec* log;
  long log_cap;
  int* log_n;
  int* log_fate;
};

__device__ __forceinline__ void atomic_add_f64(double* p, double v) {
  unsafeAtomicAdd(p, v);
}

template <bool LOG>
__global__ void __launch_bounds__(256) k_transport(TransportArgs a) {
  const DevGeom& G = a.G;
  const int lane = threadIdx.x & 63;
  const unsigned long long lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

  // per-lane track state
  bool alive = false;
  V3 x{0, 0, 0}, v{0, 0, 0};
  double E = 0, nl = 0, safety = 0;
  double mpe = 0, mco = 0, mpp = 0;
  int mat_cached = -1;
  int T = -1, tbase = 0, event = 0, zero = 0;
  long steps = 0;
  uint32_t key = 0;
  Philox rs;
  // pending annihilation photons of this lane's last primary
  int pending = 0;
  V3 px{0, 0, 0}, pw{0, 0, 0};
  long prim = 0;
  int sub = 0;
  long nrec = 0;
  // counters
  unsigned c_steps = 0, c_pe = 0, c_co = 0, c_pair = 0, c_cross = 0, c_esc = 0, c_cut = 0, c_push = 0,
           c_stuck = 0, c_trunc = 0, c_tracks = 0, c_short = 0, c_invalid = 0;
  NavCount nc{};
  bool queue_open = true;

  for (;;) {
    // ---- start a track on lanes without one --------------------------------
    bool start = false;
    if (!alive && pending > 0) {
      sub = 3 - pending;
      pending--;
      x = px;
      v = (sub == 1) ? pw : V3{-pw.x, -pw.y, -pw.z};
      E = kMe;
      key = (key & ~3u) | (uint32_t)sub;
      start = true;
    }
    bool need = !alive && !start;
    if (queue_open) {
      unsigned long long mask = __ballot(need);
      if (mask) {
        int cnt = __popcll(mask);
        int leader = __ffsll((long long)mask) - 1;
        unsigned long long base = 0;
        if (lane == leader) base = atomicAdd(a.queue, (unsigned long long)cnt);
        base = __shfl(base, leader);
        if (base + cnt >= (unsigned long long)a.n) queue_open = false;
        if (need) {
          unsigned long long idx = base + __popcll(mask & lt_mask);
          if (idx < (unsigned long long)a.n) {
            prim = (long)idx;
            sub = 0;
            x = V3{a.pos[3 * prim], a.pos[3 * prim + 1], a.pos[3 * prim + 2]};
            v = V3{a.dir[3 * prim], a.dir[3 * prim + 1], a.dir[3 * prim + 2]};
            E = a.energy[prim];
            event = a.event[prim];
            key = ((uint32_t)a.prim_id[prim]) << 2;
            int g = a.geom_default;
            bool ok = event >= 0 && event < a.n_events;
            if (ok && a.event_geom) g = a.event_geom[event];
            ok = ok && g >= 0 && g < a.n_geoms && E > 0 && isfinite(E) && isfinite(x.x) &&
                 isfinite(x.y) && isfinite(x.z) && isfinite(v.x) && isfinite(v.y) && isfinite(v.z);
            if (ok) {
              tbase = a.geom_tbase[g];
              start = true;
            } else {
              c_invalid++;
            }
          }
        }
      }
    }
    if (!__any(alive || start)) break;
    if (start) {
      // every track is located from the world of its geometry (touchable tbase)
      c_tracks++;
      nrec = 0;
      rng_start(rs, a.seed, (uint32_t)event, key);
      T = locate(G, tbase, x, true, v, nc);
      if (T < 0) {
        atomic_add_f64(a.esc_ev + event, E);
        c_esc++;
        if (LOG) {
          a.log_n[3 * prim + sub] = 0;
          a.log_fate[3 * prim + sub] = GNAV_FATE_ESCAPED;
        }
      } else {
        nl = -log(rng_next(rs));
        alive = true;
        zero = 0;
        steps = 0;
        safety = 0.0;
        mat_cached = -1;
      }
    }
    if (!alive) continue;

    // ---- one transport step ------------------------------------------------
    int fate = 0;
    if (E < a.ecut) {
      atomic_add_f64(a.edep_t + T, E);
      atomic_add_f64(a.edep_ev + event, E);
      c_cut++;
      fate = GNAV_FATE_CUTOFF;
    } else if (steps >= a.max_steps) {
      c_trunc++;
      fate = GNAV_FATE_TRUNCATED;
    } else {
      int mat = G.lv_mat[G.t_lv[T]];
      if (mat != mat_cached) {
        mu_lookup(G, mat, E, mpe, mco, mpp);
        mat_cached = mat;
      }
      double mu = mpe + mco + mpp;
      double s_phys = mu > 0 ? nl / mu : kInf;
      bool phys;
      double s_geo = kInf;
      int lim = kLimMother;
      if (s_phys < safety - kTol) {
        phys = true;
        c_short++;
      } else {
        V3 pl, vl;
        touchable_frame(G, T, x, v, pl, vl);
        double saf;
        s_geo = compute_step(G, G.t_lv[T], pl, vl, lim, saf, nc);
        safety = saf;
        phys = s_phys <= s_geo;
      }
      steps++;
      c_steps++;
      if (phys) {
        x = V3{x.x + s_phys * v.x, x.y + s_phys * v.y, x.z + s_phys * v.z};
        safety -= s_phys;
        zero = 0;
        double u = rng_next(rs) * mu;
        if (u < mpe) {
          atomic_add_f64(a.edep_t + T, E);
          atomic_add_f64(a.edep_ev + event, E);
          c_pe++;
          if (LOG && nrec < a.log_cap) {
            a.log[(3 * prim + sub) * a.log_cap + nrec] = gnav_logrec{T - tbase, kLimPE, s_phys, E, 0.0};
          }
          nrec++;
          fate = GNAV_FATE_ABSORBED;
        } else if (u < mpe + mco) {
          double eps, onecost, sint2;
          compton_sample(E, rs, eps, onecost, sint2);
          double phi = kTwoPi * rng_next(rs);
          rotate_dir(v, 1.0 - onecost, sqrt(sint2), phi);
          double dep = E * (1.0 - eps);
          E = eps * E;
          mat_cached = -1;
          atomic_add_f64(a.edep_t + T, dep);
          atomic_add_f64(a.edep_ev + event, dep);
          c_co++;
          if (LOG && nrec < a.log_cap) {
            a.log[(3 * prim + sub) * a.log_cap + nrec] =
                gnav_logrec{T - tbase, kLimCompton, s_phys, dep, E};
          }
          nrec++;
          nl = -log(rng_next(rs));
        } else {
          double dep = E - 2.0 * kMe;
          atomic_add_f64(a.edep_t + T, dep);
          atomic_add_f64(a.edep_ev + event, dep);
          c_pair++;
          double u1 = rng_next(rs), u2 = rng_next(rs);
          double ct = 1.0 - 2.0 * u1;
          double st = 2.0 * sqrt(u1 * (1.0 - u1));
          double ph = kTwoPi * u2;
          pw = V3{st * cos(ph), st * sin(ph), ct};
          px = x;
          pending = 2;
          if (LOG && nrec < a.log_cap) {
            a.log[(3 * prim + sub) * a.log_cap + nrec] = gnav_logrec{T - tbase, kLimPair, s_phys, dep, 0.0};
          }
          nrec++;
          fate = GNAV_FATE_PAIR;
        }
      } else {
        x = V3{x.x + s_geo * v.x, x.y + s_geo * v.y, x.z + s_geo * v.z};
        if (mu > 0) {
          nl = nl - s_geo * mu;
          if (nl < 0) nl = 0;
        }
        if (LOG && nrec < a.log_cap) {
          a.log[(3 * prim + sub) * a.log_cap + nrec] = gnav_logrec{T - tbase, lim, s_geo, 0.0, E};
        }
        nrec++;
        c_cross++;
        safety = 0.0;
        zero = (s_geo < kTol) ? zero + 1 : 0;
        if (zero >= kZeroKill) {
          atomic_add_f64(a.edep_t + T, E);
          atomic_add_f64(a.edep_ev + event, E);
          c_stuck++;
          fate = GNAV_FATE_STUCK;
        } else {
          if (zero > 0 && zero % kZeroPush == 0) {
            x = V3{x.x + 100.0 * kTol * v.x, x.y + 100.0 * kTol * v.y, x.z + 100.0 * kTol * v.z};
            c_push++;
          }
          int nt = relocate(G, T, x, v, lim, nc);
          if (nt < 0) {
            atomic_add_f64(a.esc_ev + event, E);
            c_esc++;
            fate = GNAV_FATE_ESCAPED;
          } else {
            T = nt;
          }
        }
      }
    }
    if (fate != 0) {
      alive = false;
      if (LOG) {
        a.log_n[3 * prim + sub] = (int)(nrec > 0x7fffffff ? 0x7fffffff : nrec);
        a.log_fate[3 * prim + sub] = fate;
      }
    }
  }

  // ---- flush counters: wave reduction, one atomic per counter per wave ----
  unsigned vals[GNAV_NCOUNTERS] = {c_steps, c_pe,    c_co,    c_pair,  c_cross,    c_esc,
                                   c_cut,   c_push,  c_stuck, c_trunc, c_tracks,   c_short,
                                   nc.dist_in, nc.dist_out, nc.inside, nc.nodes, c_invalid};
#pragma unroll
  for (int c = 0; c < GNAV_NCOUNTERS; c++) {
    unsigned long long s = vals[c];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0 && s) atomicAdd(a.counters + c, s);
  }
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
                       const double* dir, const int* touch, double* step, int* lim, int* next, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_step, dim3(grid_for(n, 256)), dim3(256), 0, st, G, W, tbase, tcount, n, pos, dir, touch,
                     step, lim, next);
  return hipGetLastError();
}

hipError_t launch_safety(const DevGeom& G, int W, int tbase, int tcount, long n, const double* pos,
                         const int* touch, double* out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_safety, dim3(grid_for(n, 256)), dim3(256), 0, st, G, W, tbase, tcount, n, pos, touch,
                     out);
  return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t words, hipStream_t st) {
  if (words == 0) return hipSuccess;
  unsigned blocks = (unsigned)std::min<size_t>((words + 255) / 256, 4096);
  hipLaunchKernelGGL(k_zero_words, dim3(blocks), dim3(256), 0, st, (unsigned long long*)p, words);
  return hipGetLastError();
}

hipError_t launch_transport(const TransportLaunch& L, hipStream_t st) {
  TransportArgs a;
  a.G = L.G;
  a.n = L.n;
  a.event = L.event;
  a.prim_id = L.prim_id;
  a.pos = L.pos;
  a.dir = L.dir;
  a.energy = L.energy;
  a.event_geom = L.event_geom;
  a.geom_default = L.geom_default;
  a.geom_tbase = L.geom_tbase;
  a.n_geoms = L.n_geoms;
  a.n_events = L.n_events;
  a.seed = L.seed;
  a.ecut = L.ecut;
  a.max_steps = L.max_steps;
  a.edep_t = L.edep_t;
  a.edep_ev = L.edep_ev;
  a.esc_ev = L.esc_ev;
  a.counters = L.counters;
  a.queue = L.queue;
  a.log = L.log;
  a.log_cap = L.log_cap;
  a.log_n = L.log_n;
  a.log_fate = L.log_fate;
  hipLaunchKernelGGL(k_reset_u64, dim3(1), dim3(64), 0, st, L.queue, 1);
  if (L.n <= 0) return hipGetLastError();
  dim3 grid(L.grid), block(L.block);
  if (L.log) hipLaunchKernelGGL(k_transport<true>, grid, block, 0, st, a);
  else hipLaunchKernelGGL(k_transport<false>, grid, block, 0, st, a);
  return hipGetLastError();
}

}  // namespace gnav

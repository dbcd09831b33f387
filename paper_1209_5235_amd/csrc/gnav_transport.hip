// gnav_transport.hip -- the persistent gamma transport kernel for gfx950
// (wave64), built once per track-pool size (GNAV_POOL slots per block: 64,
// 128 or 256), each build in its own namespace, plus a 64-slot build for
// geometries made of boxes placed without rotation (GNAV_AXIS_BOXES,
// namespace pool64_axis_boxes) and, per pool size, a build that also
// handles sphere sections (GNAV_SPHERES, namespaces pool*_spheres).
//
// Transport follows Sec. 3.1: each photon draws an Exp(1) optical depth
// (Alg. 1, steps 1-2), spends it boundary to boundary (S_j update, Eq. 6)
// and interacts where it runs out (T = t_{j-1} + (Y - S_{j-1}) / mu_j,
// Eq. 7); after a Compton scatter a new depth is drawn.  Each block keeps a
// pool of tracks in LDS and runs rounds of phases (refill, navigate, step,
// interact); before each phase the slots that need it are compacted into a
// dense work list so the lanes of a wave follow one code path (the
// divergence Sec. 5 names, handled by compaction in LDS rather than by a
// separate compaction pass).  Idle slots refill from a device work queue
// and from a block stack of annihilation photons.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "gnav_device.h"
#include "gnav_internal.h"
#include "gnav_learned.h"
#include "gnav_physics.h"

#ifndef GNAV_POOL
#define GNAV_POOL 256
#endif
#define GNAV_CAT2(a, b) a##b
#define GNAV_CAT(a, b) GNAV_CAT2(a, b)
#if defined(GNAV_AXIS_BOXES)
#define GNAV_POOL_NS GNAV_CAT(GNAV_CAT(pool, GNAV_POOL), _axis_boxes)
#elif defined(GNAV_SPHERES)
#define GNAV_POOL_NS GNAV_CAT(GNAV_CAT(pool, GNAV_POOL), _spheres)
#else
#define GNAV_POOL_NS GNAV_CAT(pool, GNAV_POOL)
#endif

static_assert(GNAV_POOL == 64 || GNAV_POOL == 128 || GNAV_POOL == 256, "track pool of 64, 128 or 256 slots");

namespace gnav {
namespace GNAV_POOL_NS {

// Occupancy target for the transport kernel (waves per SIMD, settable at
// build time; 0 leaves register allocation to the compiler).  Two waves per
// SIMD (two 256-slot blocks per compute unit) caps a wave at 256 registers,
// VGPRs and AGPRs together, which the learned-order instantiation would
// otherwise exceed.
// The axis-aligned box build needs fewer registers: with a smaller block
// stack and deposit cache (below) its 64-slot block fits in 13 KB of LDS and
// three waves per SIMD are resident (24 spilled registers; measured 3 %
// faster than two).
#ifndef GNAV_TRANSPORT_WAVES
#ifdef GNAV_AXIS_BOXES
#define GNAV_TRANSPORT_WAVES 3
#else
#define GNAV_TRANSPORT_WAVES 2
#endif
#endif
#if GNAV_TRANSPORT_WAVES > 0
#define GNAV_TRANSPORT_ATTR __attribute__((amdgpu_waves_per_eu(GNAV_TRANSPORT_WAVES)))
#else
#define GNAV_TRANSPORT_ATTR
#endif

// ---------------------------------------------------------------------------
// Block track pool.  Each block owns kPool track slots held in LDS as
// structure of arrays.  One loop iteration runs four block-wide phases:
//   refill   - empty slots take a pending annihilation photon or a queued
//              primary (one queue atomic per wave);
//   navigate - slots that start a track or crossed a boundary relocate;
//   step     - slots ready to move compute mu, the safety shortcut or a
//              ComputeStep, and advance;
//   interact - slots whose step ended in an interaction sample it.
// Before each phase the slots that need it are compacted into a dense work
// list with wave ballots and a block prefix sum (optionally bucketed by a
// small key: the mother's solid type for steps, the process for
// interactions), so the lanes of a wave run the same code path.
// ---------------------------------------------------------------------------

constexpr int kPool = GNAV_POOL;
constexpr int kWaves = kPool / 64;
#ifdef GNAV_AXIS_BOXES
constexpr int kStack = 16;       // block stack of annihilation photons (entries)
constexpr int kDep = kPool;      // block cache of touchable deposits
constexpr int kDepProbes = 4;    // entries a touchable may take (hashed group)
// interact passes with fewer slots due than this wait a round (eighths of the
// pool, settable at build time)
#ifndef GNAV_INT_HOLD_EIGHTHS
#define GNAV_INT_HOLD_EIGHTHS 3
#endif
constexpr int kIntHold = (GNAV_INT_HOLD_EIGHTHS * kPool) / 8;
#else
constexpr int kStack = 64;
constexpr int kDep = 4 * kPool;
constexpr int kDepProbes = 1;    // direct mapped
#ifndef GNAV_INT_HOLD_EIGHTHS
#define GNAV_INT_HOLD_EIGHTHS 2
#endif
constexpr int kIntHold = (GNAV_INT_HOLD_EIGHTHS * kPool) / 8;
#endif

// counters summed per block in LDS (the work counters of counting launches,
// from GNAV_C_DIST_IN_BY on, go from each wave to the tally directly)
constexpr int kBlockCounters = GNAV_C_SCORED + 1;
static_assert(kBlockCounters <= kPool, "one counter per thread at the block's start and end");

// slot status
enum : int { kEmpty = 0, kNav = 1, kStep = 2, kInt = 3 };
// process codes for kInt
enum : int { kProcPE = 0, kProcCompton = 1, kProcPair = 2 };

struct Pool {
  double x[kPool], y[kPool], z[kPool], vx[kPool], vy[kPool], vz[kPool];
  double E[kPool], nl[kPool], saf[kPool], mu[kPool], wmu[kPool];
  int T[kPool], lvk[kPool], tbase[kPool], event[kPool], key[kPool], draw[kPool];
  int status[kPool];  // kEmpty / kNav / kStep / kInt
  int aux[kPool];     // kNav: navigation mode | lim << 2 ; kInt: process
  int zero_steps[kPool];  // zero-step count (low 8 bits) | steps << 8
  int imu_mat[kPool];     // table node | cached material << 9 (material + 1, 0 = none)
  int prim[kPool];
  int sub_pend[kPool];    // photon index (0..2) | pending annihilation photons << 4
  int nrec[kPool];
  unsigned cnt_a[kPool];  // Compton scatters | shortcuts << 16
  unsigned cnt_b[kPool];  // crossings | pushes << 24
  double dep[kPool];   // deposits of the slot's current track, added to its event at the end
  // annihilation photons waiting for any free slot of the block (a stack)
  double sx[kStack], sy[kStack], sz[kStack], svx[kStack], svy[kStack], svz[kStack];
  int sev[kStack], skey[kStack], stb[kStack], sprim[kStack];
  int sn;              // valid stack entries
  int dkey[kDep];      // touchable of a cached deposit sum (-1: free)
  double dval[kDep];
  int list[kPool];
  int wcnt[16 * kWaves];
  int total[16];
  unsigned long long cnt[kBlockCounters];
  long qr[4];          // block-claimed primaries not yet started: [qr0, qr1) then [qr2, qr3)
  int qopen;           // the device queue may still hold primaries
  int any_alive;
};

// Dense work list of the slots with `flag`, bucketed by `key` in [0, K):
// list entries of bucket 0 first, then bucket 1, ...  Returns the count
// (block uniform).  Must be called by every thread of the block.
template <int K>
__device__ __forceinline__ int compact(Pool& P, bool flag, int key) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  unsigned long long my_mask = 0;
#pragma unroll
  for (int b = 0; b < K; b++) {
    unsigned long long m = __ballot(flag && key == b);
    if (flag && key == b) my_mask = m;
    if (lane == 0) P.wcnt[b * kWaves + w] = __popcll(m);
  }
  __syncthreads();
  if (threadIdx.x < K) {
    int t = 0;
#pragma unroll
    for (int ww = 0; ww < kWaves; ww++) t += P.wcnt[threadIdx.x * kWaves + ww];
    P.total[threadIdx.x] = t;
  }
  __syncthreads();
  int n = 0;
#pragma unroll
  for (int b = 0; b < K; b++) n += P.total[b];
  if (flag) {
    int base = 0;
    for (int b = 0; b < key; b++) base += P.total[b];
    for (int ww = 0; ww < w; ww++) base += P.wcnt[key * kWaves + ww];
    P.list[base + __popcll(my_mask & lt)] = threadIdx.x;
  }
  __syncthreads();
  return n;
}

static_assert((kDep & (kDep - 1)) == 0 && kDepProbes <= kDep, "deposit cache: power-of-two entries");

// Add d to cache entry h if touchable T owns it or can claim it.
__device__ __forceinline__ bool dep_try(Pool& P, int h, int T, double d) {
  int owner = P.dkey[h];
  if (owner == -1) {
    owner = atomicCAS(&P.dkey[h], -1, T);
    if (owner == -1) owner = T;
  }
  if (owner != T) return false;
  atomicAdd(&P.dval[h], d);
  return true;
}

// Deposit d in touchable T: summed in the block's LDS cache when T owns (or
// can claim) one of its candidate entries, else added to the device tally
// directly; the cache is added to the tally when the block ends.  A claimed
// entry keeps its touchable until the block ends and the candidates are tried
// in a fixed order, so a touchable holds at most one entry.  One candidate:
// T mod kDep, which gives consecutive touchables (the phi segments of a ring)
// distinct entries.  Several: an aligned group picked by a multiplicative
// (Fibonacci) hash of T, so that touchables a fixed stride apart (the cells
// of stacked layers) do not all fall on a few entries.
__device__ __forceinline__ void deposit_t(Pool& P, const TransportArgs& a, int T, double d) {
  int h;
  if constexpr (kDepProbes == 1) h = T & (kDep - 1);
  else h = (int)(((unsigned)T * 2654435769u) >> (32 - __builtin_ctz(kDep)));
#pragma unroll
  for (int k = 0; k < kDepProbes; k++)
    if (dep_try(P, h ^ k, T, d)) return;
  atomic_add_f64(a.edep_t + T, d);
}

template <bool LOG>
__device__ __forceinline__ void end_track(Pool& P, const TransportArgs& a, int s, int fate, int steps) {
  P.status[s] = kEmpty;
  if (P.dep[s] != 0.0) atomic_add_f64(a.edep_ev + P.event[s], P.dep[s]);
  int slot = fate == GNAV_FATE_ABSORBED ? GNAV_C_PE
           : fate == GNAV_FATE_PAIR     ? GNAV_C_PAIR
           : fate == GNAV_FATE_ESCAPED  ? GNAV_C_ESCAPED
           : fate == GNAV_FATE_CUTOFF   ? GNAV_C_CUTOFF
           : fate == GNAV_FATE_STUCK    ? GNAV_C_STUCK
                                        : GNAV_C_TRUNCATED;
  atomicAdd(&P.cnt[slot], 1ull);
  if (steps) atomicAdd(&P.cnt[GNAV_C_STEPS], (unsigned long long)steps);
  unsigned ca = P.cnt_a[s], cb = P.cnt_b[s];
  if (ca & 0xFFFF) atomicAdd(&P.cnt[GNAV_C_COMPTON], (unsigned long long)(ca & 0xFFFF));
  if (ca >> 16) atomicAdd(&P.cnt[GNAV_C_SHORTCUTS], (unsigned long long)(ca >> 16));
  if (cb & 0xFFFFFF) atomicAdd(&P.cnt[GNAV_C_CROSSINGS], (unsigned long long)(cb & 0xFFFFFF));
  if (cb >> 24) atomicAdd(&P.cnt[GNAV_C_PUSHES], (unsigned long long)(cb >> 24));
  if (LOG) {
    const long slot3 = 3L * P.prim[s] + (P.sub_pend[s] & 15);
    if (a.log_n) a.log_n[slot3] = P.nrec[s];
    if (a.log_fate) a.log_fate[slot3] = fate;
    if (a.digest) {
      a.digest[slot3].n = P.nrec[s];
      a.digest[slot3].fate = fate;
    }
  }
}

// 64-bit FNV-1a over the touchable and the code of one step record, each as
// four little-endian bytes (the per-track digest's hash).
__device__ __forceinline__ uint64_t fnv1a_record(uint64_t h, int touchable, int code) {
  const uint32_t w[2] = {(uint32_t)touchable, (uint32_t)code};
#pragma unroll
  for (int k = 0; k < 2; k++) {
#pragma unroll
    for (int b = 0; b < 4; b++) {
      h ^= (w[k] >> (8 * b)) & 0xffu;
      h *= 1099511628211ull;
    }
  }
  return h;
}

template <bool LOG>
__device__ __forceinline__ void digest_start(Pool& P, const TransportArgs& a, int s) {
  if (LOG && a.digest) {
    gnav_digest& d = a.digest[3L * P.prim[s] + (P.sub_pend[s] & 15)];
    d.hash = 14695981039346656037ull;
    d.n = 0;
    d.fate = 0;
    d.sum_step = 0.0;
    d.sum_edep = 0.0;
  }
}

template <bool LOG>
__device__ __forceinline__ void log_rec(Pool& P, const TransportArgs& a, int s, int T, int code, double step,
                                        double edep, double energy) {
  if (LOG) {
    int n = P.nrec[s];
    const long slot3 = 3L * P.prim[s] + (P.sub_pend[s] & 15);
    if (n < a.log_cap) a.log[slot3 * a.log_cap + n] = gnav_logrec{T - P.tbase[s], code, step, edep, energy};
    if (a.digest) {
      gnav_digest& d = a.digest[slot3];
      d.hash = fnv1a_record(d.hash, T - P.tbase[s], code);
      d.sum_step += step;
      d.sum_edep += edep;
    }
    P.nrec[s] = n + 1;
  }
}

// Learned order: the block gathers the features of its eligible steps here
// and the network (gnav_learned.h) writes each step's predicted candidate
// position over its class.
// Block memory of the learned order only (the other instantiations leave it
// out).
struct LearnScratch {
  uint16_t xf[kPool][6];  // bf16 features of the listed steps (mother-frame point, direction)
  uint16_t cls[kPool];    // their ordering classes in, the predicted candidate positions out
  int pred[kPool];        // predicted candidate position of each slot's next step
};
struct NoScratch {};
// Block memory of logging launches only (per-track logs and digests): the
// physics step that ended at each pending interaction.  Leaving this and the
// learned order's memory out of the other instantiations keeps the 64-slot
// box build at 12.6 KB of LDS, which twelve blocks per CU hold (at 13.1 KB
// only eleven were resident).
struct LogScratch {
  double slast[kPool];
};

template <bool LOG, bool COUNT, int ORDER, int PREC>
__global__ void __launch_bounds__(kPool) GNAV_TRANSPORT_ATTR k_transport(TransportArgs a) {
  const DevGeom& G = a.G;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const unsigned long long lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  __shared__ Pool P;
  __shared__ typename std::conditional<ORDER == kOrderLearned, LearnScratch, NoScratch>::type S;
  __shared__ typename std::conditional<LOG, LogScratch, NoScratch>::type LS;
  double* const my_pend = a.pend + ((long)blockIdx.x * kPool + tid) * 6;

  if (tid < kBlockCounters) P.cnt[tid] = 0ull;
  if (tid < 4) P.qr[tid] = 0;
  if (tid == 0) {
    P.qopen = 1;
    P.sn = 0;
  }
  P.status[tid] = kEmpty;
  P.sub_pend[tid] = 0;
  for (int i = tid; i < kDep; i += kPool) {
    P.dkey[i] = -1;
    P.dval[i] = 0.0;
  }
  NavCount<COUNT> nc;
  bool queue_open = true;
  bool int_deferred = false;  // block uniform: the interact pass was held last round
  __syncthreads();

  for (int round = 0;; round++) {
    // ---- refill: thread tid owns slot tid ---------------------------------
    {
      const int s = tid;
      bool empty = P.status[s] == kEmpty;
      int sp = P.sub_pend[s];
      int pending = sp >> 4;
      bool start = false;
      if (empty && pending > 0) {
        int sub = 3 - pending;
        P.sub_pend[s] = sub | ((pending - 1) << 4);
        P.x[s] = my_pend[0];
        P.y[s] = my_pend[1];
        P.z[s] = my_pend[2];
        double sgn = (sub == 1) ? 1.0 : -1.0;
        P.vx[s] = sgn * my_pend[3];
        P.vy[s] = sgn * my_pend[4];
        P.vz[s] = sgn * my_pend[5];
        P.E[s] = kMe;
        P.key[s] = (P.key[s] & ~3) | sub;
        start = true;
      }
      bool need = empty && !start;
      // annihilation photons parked on the block stack go to free slots first
      const int sn = P.sn;
      if (sn > 0) {
        const int w = tid >> 6;
        unsigned long long mask = __ballot(need);
        if (lane == 0) P.wcnt[w] = __popcll(mask);
        __syncthreads();
        int before = 0, n_need = 0;
#pragma unroll
        for (int ww = 0; ww < kWaves; ww++) {
          int c = P.wcnt[ww];
          if (ww < w) before += c;
          n_need += c;
        }
        if (need) {
          int rank = before + __popcll(mask & lt_mask);
          if (rank < sn) {
            const int e = sn - 1 - rank;
            P.x[s] = P.sx[e];
            P.y[s] = P.sy[e];
            P.z[s] = P.sz[e];
            P.vx[s] = P.svx[e];
            P.vy[s] = P.svy[e];
            P.vz[s] = P.svz[e];
            P.E[s] = kMe;
            P.event[s] = P.sev[e];
            P.key[s] = P.skey[e];
            P.tbase[s] = P.stb[e];
            P.prim[s] = P.sprim[e];
            P.sub_pend[s] = P.skey[e] & 3;
            start = true;
            need = false;
          }
        }
        __syncthreads();
        if (tid == 0) P.sn = sn - min(sn, n_need);
      }
      long idx = -1;
      if (a.chunk <= 0) {
        // each wave claims exactly the primaries its idle lanes need
        unsigned long long mask = queue_open ? __ballot(need) : 0ull;
        if (mask) {
          int cnt = __popcll(mask);
          int leader = __ffsll((long long)mask) - 1;
          unsigned long long base = 0;
          if (lane == leader) base = atomicAdd(a.queue, (unsigned long long)cnt);
          base = __shfl(base, leader);
          if (base + cnt >= (unsigned long long)a.n) queue_open = false;
          if (need) {
            unsigned long long q = base + __popcll(mask & lt_mask);
            if (q < (unsigned long long)a.n) idx = (long)q;
          }
        }
      } else {
        // the block claims `chunk` primaries at a time and hands them out in
        // slot order; at most two claimed ranges are open at once
        const int w = tid >> 6;
        unsigned long long mask = __ballot(need);
        if (lane == 0) P.wcnt[w] = __popcll(mask);
        __syncthreads();
        int before = 0, n_need = 0;
#pragma unroll
        for (int ww = 0; ww < kWaves; ww++) {
          int c = P.wcnt[ww];
          if (ww < w) before += c;
          n_need += c;
        }
        if (tid == 0 && P.qopen) {
          long have = (P.qr[1] - P.qr[0]) + (P.qr[3] - P.qr[2]);
          if (have < n_need) {
            long want = max((long)a.chunk, (long)n_need - have);
            long base = (long)atomicAdd(a.queue, (unsigned long long)want);
            long end = min(base + want, a.n);
            if (base + want >= a.n) P.qopen = 0;
            if (base < end) {
              if (P.qr[1] == P.qr[0]) {
                P.qr[0] = P.qr[2];
                P.qr[1] = P.qr[3];
              }
              if (P.qr[1] == P.qr[0]) {
                P.qr[0] = base;
                P.qr[1] = end;
                P.qr[2] = P.qr[3] = 0;
              } else {
                P.qr[2] = base;
                P.qr[3] = end;
              }
            }
          }
        }
        __syncthreads();
        const long r0 = P.qr[0], r1 = P.qr[1], r2 = P.qr[2], r3 = P.qr[3];
        if (need) {
          long rank = before + __popcll(mask & lt_mask);
          if (rank < r1 - r0) idx = r0 + rank;
          else if (rank - (r1 - r0) < r3 - r2) idx = r2 + rank - (r1 - r0);
        }
        __syncthreads();
        if (tid == 0) {
          long take = n_need;
          long t1 = min(take, r1 - r0);
          P.qr[0] = r0 + t1;
          take -= t1;
          long t2 = min(take, r3 - r2);
          P.qr[2] = r2 + t2;
          if (P.qr[2] == P.qr[3]) P.qr[2] = P.qr[3] = 0;
        }
      }
      if (idx >= 0) {
        // the primary at this queue position: from the claim-order copy
        // (decreasing energy) when the library built one
        V3 x, v;
        double E;
        int event, prim_id;
        if (a.claim) {
          const ClaimRec& r = a.claim[idx];
          x = V3{r.pos[0], r.pos[1], r.pos[2]};
          v = V3{r.dir[0], r.dir[1], r.dir[2]};
          E = r.energy;
          event = r.event;
          prim_id = r.prim_id;
          idx = r.index;
        } else {
          x = V3{a.pos[3 * idx], a.pos[3 * idx + 1], a.pos[3 * idx + 2]};
          v = V3{a.dir[3 * idx], a.dir[3 * idx + 1], a.dir[3 * idx + 2]};
          E = a.energy[idx];
          event = a.event[idx];
          prim_id = a.prim_id[idx];
        }
        int g = a.geom_default;
        bool ok = event >= 0 && event < a.n_events;
        if (ok && a.event_geom) g = a.event_geom[event];
        ok = ok && g >= 0 && g < a.n_geoms && E > 0 && isfinite(E) && isfinite(x.x) && isfinite(x.y) &&
             isfinite(x.z) && isfinite(v.x) && isfinite(v.y) && isfinite(v.z);
        if (ok) {
          P.x[s] = x.x;
          P.y[s] = x.y;
          P.z[s] = x.z;
          P.vx[s] = v.x;
          P.vy[s] = v.y;
          P.vz[s] = v.z;
          P.E[s] = E;
          P.event[s] = event;
          P.key[s] = prim_id << 2;
          P.tbase[s] = a.geom_tbase[g];
          P.prim[s] = (int)idx;
          P.sub_pend[s] = 0;
          start = true;
        } else {
          atomicAdd(&P.cnt[GNAV_C_INVALID], 1ull);
        }
      }
      if (start) {
        P.status[s] = kNav;
        P.aux[s] = kNavStart;
        P.T[s] = P.tbase[s];
      }
    }
    // done when no slot holds a track and no claimed or unclaimed primary is
    // left (a refill that met only invalid primaries does not end the block)
    {
      bool more = P.status[tid] != kEmpty;
      if (a.chunk <= 0) more = more || queue_open;
      else if (tid == 0) more = more || P.qopen || P.qr[1] > P.qr[0] || P.qr[3] > P.qr[2];
      if (!__syncthreads_or(more)) break;
    }

    // ---- navigate: track starts and boundary crossings --------------------
    {
      int n = compact<1>(P, P.status[tid] == kNav, 0);
      if (tid < n) {
        const int s = P.list[tid];
        const int mode = P.aux[s] & 3;
        const int lim = P.aux[s] >> 2;  // entered slot, or (exits) the face left (-1 unknown)
        V3 x{P.x[s], P.y[s], P.z[s]}, v{P.vx[s], P.vy[s], P.vz[s]};
        if (mode == kNavStart) {
          digest_start<LOG>(P, a, s);
          atomicAdd(&P.cnt[GNAV_C_TRACKS], 1ull);
          P.draw[s] = 0;
          P.dep[s] = 0.0;
          P.nrec[s] = 0;
          P.zero_steps[s] = 0;
          P.cnt_a[s] = 0;
          P.cnt_b[s] = 0;
          P.saf[s] = 0.0;
        }
        int lvk = 0;
        int nt = navigate(G, mode, P.T[s], lim, x, v, lvk, nc, mode == kNavExit ? lim : -1);
        if (nt < 0) {
          atomic_add_f64(a.esc_ev + P.event[s], P.E[s]);
          end_track<LOG>(P, a, s, GNAV_FATE_ESCAPED, P.zero_steps[s] >> 8);
        } else {
          P.T[s] = nt;
          P.lvk[s] = lvk;
          P.status[s] = kStep;
          if (mode == kNavStart) {
            Philox rs{(uint32_t)P.event[s], (uint32_t)P.key[s], 0u};
            P.nl[s] = -log(rng_next(rs, a.seed_lo, a.seed_hi));
            P.draw[s] = (int)rs.draw;
            int imu;
            double w;
            mu_index(G, P.E[s], imu, w);
            P.imu_mat[s] = imu;  // no cached material
            P.wmu[s] = w;
          }
        }
      }
      __syncthreads();
    }

    // ---- learned order: score the steps whose mother has a voxel grid -------
    // (only steps in mothers whose voxel nodes hold enough candidates on
    // average for an order to pay)
    if constexpr (ORDER == kOrderLearned) {
      bool elig = false;
      if (P.status[tid] == kStep) {
        const LRec& L = G.lv[P.lvk[tid] >> 1];
        elig = L.lclass >= 0 && L.wide;
      }
      S.pred[tid] = -1;
      int n = compact<1>(P, elig, 0);
      // Score only when a full 16-row tile is due: the out-of-line call saves
      // and restores the live registers of the loop through scratch memory,
      // which a few rows do not repay.  Unscored steps take the nearest
      // enclosing cylinder first, as in the bound order; results are the same.
      if (n >= 16) {
        // features of listed step i: the point in the mother frame over the
        // voxel grid's half size (centred on the grid), and the direction
        if (tid < n) {
          const int s = P.list[tid];
          const int lvk = P.lvk[s];
          V3 x{P.x[s], P.y[s], P.z[s]}, v{P.vx[s], P.vy[s], P.vz[s]};
          V3 pl, vl;
          touchable_frame(G, P.T[s], lvk & 1, x, v, pl, vl);
          learned_features(G.lv[lvk >> 1], pl, vl, a.mlp.n_class, S.xf[tid], &S.cls[tid]);
        }
        __syncthreads();
        learned_predict<kWaves>(a.mlp, S.xf, S.cls, n);
        __syncthreads();
        if (tid < n) S.pred[P.list[tid]] = S.cls[tid];
        if (tid == 0) atomicAdd(&P.cnt[GNAV_C_SCORED], (unsigned long long)n);
      }
      __syncthreads();
    }

    // ---- step: mu, safety shortcut or ComputeStep, advance ------------------
    {
      // bucket the step work by solid family and daughters, or, every
      // sort_period-th round, by the current logical volume (16 ranges of LV id)
      const bool by_volume = a.sort_period > 0 && round % a.sort_period == 0;
      int key = 0;
      if (P.status[tid] == kStep) {
        const int lv = P.lvk[tid] >> 1;
        if (by_volume) {
          key = (int)(((long)lv * 16) / a.n_lv);
        } else {
          const LRec& L = G.lv[lv];
          key = (L.info & 3) | (L.dau_cnt > 0 ? 4 : 0);
        }
      }
      int n = by_volume ? compact<16>(P, P.status[tid] == kStep, key)
                        : compact<8>(P, P.status[tid] == kStep, key);
      if (tid < n) {
        const int s = P.list[tid];
        const int T = P.T[s];
        const int lvk = P.lvk[s];
        const LRec& L = G.lv[lvk >> 1];
        double E = P.E[s];
        int zs = P.zero_steps[s];
        int steps = zs >> 8;
        int zero = zs & 0xFF;
        if (E < a.ecut) {
          deposit_t(P, a, T, E);
          P.dep[s] += E;
          end_track<LOG>(P, a, s, GNAV_FATE_CUTOFF, steps);
        } else if (steps >= a.max_steps) {
          end_track<LOG>(P, a, s, GNAV_FATE_TRUNCATED, steps);
        } else {
          const int mat = L.mat;
          int im = P.imu_mat[s];
          const int imu = im & 511;
          const double wmu = P.wmu[s];
          double mu;
          if ((im >> 9) != mat + 1) {
            double pe, co, pp;
            mu_parts(G, mat, imu, wmu, E, pe, co, pp);
            mu = pe + co + pp;
            P.mu[s] = mu;
            P.imu_mat[s] = imu | ((mat + 1) << 9);
          } else {
            mu = P.mu[s];
          }
          double nl = P.nl[s];
          double safety = P.saf[s];
          V3 x{P.x[s], P.y[s], P.z[s]}, v{P.vx[s], P.vy[s], P.vz[s]};
          double s_phys = mu > 0 ? nl / mu : kInf;
          bool phys;
          double s_geo = kInf;
          int lim = kLimMother;
          int exit_face = -1;
          if (s_phys < safety - kTol) {
            phys = true;
            P.cnt_a[s] += 1u << 16;
          } else {
            V3 pl, vl;
            touchable_frame(G, T, lvk & 1, x, v, pl, vl);
            if (COUNT) nc.levels(trec_depth(G.t[T]));
            double saf;
            int2 nd;
            int pred = -1;
            if constexpr (ORDER == kOrderLearned) pred = S.pred[s];
            s_geo = compute_step_p<COUNT, ORDER, PREC>(G, L, lvk >> 1, pl, vl, lim, saf, nc, pred, &nd);
            safety = saf;
            phys = s_phys <= s_geo;
            // the face a box is left through, for the neighbour shortcut of the relocation
            if (!phys && lim == kLimMother && (L.info & 15) == kBox)
              exit_face = box_face(L.par, V3{pl.x + s_geo * vl.x, pl.y + s_geo * vl.y, pl.z + s_geo * vl.z});
            // crossing recorder: a daughter-limited step from a node with 2+ candidates
            if (a.rec && !phys && lim >= 0 && nd.y >= 2 && L.lclass >= 0) {
              int label = -1;
              for (int c = 0; c < nd.y && c < 64; c++)
                if (G.vox_cand[nd.x + c] == lim) label = c;
              if (label >= 0) {
                unsigned long long ri = atomicAdd(a.rec_count, 1ull);
                if (ri < (unsigned long long)a.rec_cap) {
                  gnav_crossing cr;
                  cr.cls = L.lclass;
                  const double pc[3] = {pl.x, pl.y, pl.z};
#pragma unroll
                  for (int ax = 0; ax < 3; ax++) {
                    double half = 0.5 * L.n[ax] * L.vw[ax];
                    cr.x[ax] = (float)((pc[ax] - (L.vlo[ax] + half)) / half);
                  }
                  cr.v[0] = (float)vl.x;
                  cr.v[1] = (float)vl.y;
                  cr.v[2] = (float)vl.z;
                  cr.label = label;
                  a.rec[ri] = cr;
                }
              }
            }
          }
          steps++;
          if (phys) {
            P.x[s] = x.x + s_phys * v.x;
            P.y[s] = x.y + s_phys * v.y;
            P.z[s] = x.z + s_phys * v.z;
            P.saf[s] = safety - s_phys;
            P.zero_steps[s] = steps << 8;
            // process choice: the first draw after the step (u mu against the partial sums)
            double pe, co, pp;
            mu_parts(G, mat, imu, wmu, E, pe, co, pp);
            Philox rs{(uint32_t)P.event[s], (uint32_t)P.key[s], (uint32_t)P.draw[s]};
            double u = rng_next(rs, a.seed_lo, a.seed_hi) * mu;
            P.draw[s] = (int)rs.draw;
            P.aux[s] = u < pe ? kProcPE : (u < pe + co ? kProcCompton : kProcPair);
            if constexpr (LOG) LS.slast[s] = s_phys;
            P.status[s] = kInt;
          } else {
            // the pure FP32 form steps past the boundary by its surface band, so
            // the FP64 relocation sees the point on the far side of the face
            const double s_adv = PREC == kPrecPure ? s_geo + 2.0 * (double)kHalfTolF : s_geo;
            P.x[s] = x.x + s_adv * v.x;
            P.y[s] = x.y + s_adv * v.y;
            P.z[s] = x.z + s_adv * v.z;
            if (mu > 0) {
              nl = nl - s_adv * mu;
              if (nl < 0) nl = 0;
              P.nl[s] = nl;
            }
            log_rec<LOG>(P, a, s, T, lim, s_adv, 0.0, E);
            P.cnt_b[s] += 1u;
            P.saf[s] = 0.0;
            // zero-length steps and the push that ends a run of them, on the
            // length scale of the surface band of the distance arithmetic
            constexpr double kZeroLen = PREC == kPrecPure ? 2.0 * kHalfTolF : kTol;
            constexpr double kPushLen = PREC == kPrecPure ? 10.0 * kZeroLen : 100.0 * kTol;
            zero = (s_geo < kZeroLen) ? zero + 1 : 0;
            P.zero_steps[s] = (steps << 8) | zero;
            if (zero >= kZeroKill) {
              deposit_t(P, a, T, E);
              P.dep[s] += E;
              end_track<LOG>(P, a, s, GNAV_FATE_STUCK, steps);
            } else {
              if (zero > 0 && zero % kZeroPush == 0) {
                P.x[s] = P.x[s] + kPushLen * v.x;
                P.y[s] = P.y[s] + kPushLen * v.y;
                P.z[s] = P.z[s] + kPushLen * v.z;
                P.cnt_b[s] += 1u << 24;
              }
              // relocation happens in the next iteration's navigation phase
              P.aux[s] = lim >= 0 ? (kNavEnter | (lim << 2)) : (kNavExit | (exit_face << 2));
              P.status[s] = kNav;
            }
          }
        }
      }
      __syncthreads();
    }

    // ---- interact: photoelectric, Compton, pair ------------------------------
    {
      int n = compact<3>(P, P.status[tid] == kInt, P.aux[tid]);
      // With few slots due (under a quarter of the pool, three eighths in the
      // axis-aligned box build: measured best for each), hold them for one
      // round so the next pass serves more of them at once; a held track only
      // waits, so the results do not change.
      if (n < kIntHold && !int_deferred) { int_deferred = true; n = 0; }
      else int_deferred = false;
      if (tid < n) {
        const int s = P.list[tid];
        const int proc = P.aux[s];
        const int T = P.T[s];
        const int event = P.event[s];
        const double E = P.E[s];
        double sl = 0.0;
        if constexpr (LOG) sl = LS.slast[s];
        const int steps = P.zero_steps[s] >> 8;
        Philox rs{(uint32_t)event, (uint32_t)P.key[s], (uint32_t)P.draw[s]};
        if (proc == kProcPE) {
          deposit_t(P, a, T, E);
          P.dep[s] += E;
          log_rec<LOG>(P, a, s, T, kLimPE, sl, E, 0.0);
          end_track<LOG>(P, a, s, GNAV_FATE_ABSORBED, steps);
        } else if (proc == kProcCompton) {
          double eps, onecost, sint2;
          compton_sample(E, rs, a.seed_lo, a.seed_hi, eps, onecost, sint2);
          double phi = kTwoPi * rng_next(rs, a.seed_lo, a.seed_hi);
          V3 v{P.vx[s], P.vy[s], P.vz[s]};
          rotate_dir(v, 1.0 - onecost, sqrt(sint2), phi);
          P.vx[s] = v.x;
          P.vy[s] = v.y;
          P.vz[s] = v.z;
          double dep = E * (1.0 - eps);
          double E2 = eps * E;
          P.E[s] = E2;
          int imu;
          double w;
          mu_index(G, E2, imu, w);
          P.imu_mat[s] = imu;  // cached mu invalid
          P.wmu[s] = w;
          deposit_t(P, a, T, dep);
          P.dep[s] += dep;
          P.cnt_a[s] += 1u;
          log_rec<LOG>(P, a, s, T, kLimCompton, sl, dep, E2);
          P.nl[s] = -log(rng_next(rs, a.seed_lo, a.seed_hi));
          P.draw[s] = (int)rs.draw;
          P.status[s] = kStep;
        } else {
          double dep = E - 2.0 * kMe;
          deposit_t(P, a, T, dep);
          P.dep[s] += dep;
          double u1 = rng_next(rs, a.seed_lo, a.seed_hi), u2 = rng_next(rs, a.seed_lo, a.seed_hi);
          double ct = 1.0 - 2.0 * u1;
          double st = 2.0 * sqrt(u1 * (1.0 - u1));
          double ph = kTwoPi * u2;
          const double wx = st * cos(ph), wy = st * sin(ph), wz = ct;
          // both photons onto the block stack, so two free slots can take them
          // at once; when it is full, this slot tracks them one after the other
          const int e = atomicAdd(&P.sn, 2);
          if (e + 2 <= kStack) {
#pragma unroll
            for (int j = 0; j < 2; j++) {
              const double sg = j == 0 ? 1.0 : -1.0;
              P.sx[e + j] = P.x[s];
              P.sy[e + j] = P.y[s];
              P.sz[e + j] = P.z[s];
              P.svx[e + j] = sg * wx;
              P.svy[e + j] = sg * wy;
              P.svz[e + j] = sg * wz;
              P.sev[e + j] = event;
              P.skey[e + j] = (P.key[s] & ~3) | (j + 1);
              P.stb[e + j] = P.tbase[s];
              P.sprim[e + j] = P.prim[s];
            }
          } else {
            atomicSub(&P.sn, 2);
            double* pd = a.pend + ((long)blockIdx.x * kPool + s) * 6;
            pd[0] = P.x[s];
            pd[1] = P.y[s];
            pd[2] = P.z[s];
            pd[3] = wx;
            pd[4] = wy;
            pd[5] = wz;
            P.sub_pend[s] = (P.sub_pend[s] & 15) | (2 << 4);
          }
          log_rec<LOG>(P, a, s, T, kLimPair, sl, dep, 0.0);
          end_track<LOG>(P, a, s, GNAV_FATE_PAIR, steps);
        }
      }
      __syncthreads();
    }
  }

  // ---- flush the deposit cache and the counters ---------------------------
  __syncthreads();
  for (int i = tid; i < kDep; i += kPool)
    if (P.dkey[i] >= 0 && P.dval[i] != 0.0) atomic_add_f64(a.edep_t + P.dkey[i], P.dval[i]);
  if (COUNT) {
    constexpr int F = GNAV_NFAMILIES;
    constexpr int kNV = 6 + 4 * F;
    unsigned vals[kNV];
    int slots[kNV];
    vals[0] = nc.total(nc.din) - nc.dist_in32;
    slots[0] = GNAV_C_DIST_IN;
    vals[1] = nc.total(nc.dout);
    slots[1] = GNAV_C_DIST_OUT;
    vals[2] = nc.total(nc.dins);
    slots[2] = GNAV_C_INSIDE;
    vals[3] = nc.nodes;
    slots[3] = GNAV_C_VOXEL_NODES;
    vals[4] = nc.dist_in32;
    slots[4] = GNAV_C_DIST_IN_F32;
    vals[5] = nc.frames;
    slots[5] = GNAV_C_FRAME_MAPS;
#pragma unroll
    for (int f = 0; f < F; f++) {
      vals[6 + f] = nc.din[f];
      slots[6 + f] = GNAV_C_DIST_IN_BY + f;
      vals[6 + F + f] = nc.dout[f];
      slots[6 + F + f] = GNAV_C_DIST_OUT_BY + f;
      vals[6 + 2 * F + f] = nc.dsaf[f];
      slots[6 + 2 * F + f] = GNAV_C_SAFETY_BY + f;
      vals[6 + 3 * F + f] = nc.dins[f];
      slots[6 + 3 * F + f] = GNAV_C_INSIDE_BY + f;
    }
#pragma unroll
    for (int c = 0; c < kNV; c++) {
      unsigned long long sum = vals[c];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
      if (lane == 0 && sum) atomicAdd(a.counters + slots[c], sum);
    }
  }
  __syncthreads();
  if (tid < kBlockCounters && P.cnt[tid]) atomicAdd(a.counters + tid, P.cnt[tid]);
}

hipError_t launch(const TransportLaunch& L, hipStream_t st) {
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
  a.seed_lo = (uint32_t)L.seed;
  a.seed_hi = (uint32_t)(L.seed >> 32);
  a.ecut = L.ecut;
  a.max_steps = (int)std::min<long>(L.max_steps, 0x7fffffff);
  a.edep_t = L.edep_t;
  a.edep_ev = L.edep_ev;
  a.esc_ev = L.esc_ev;
  a.counters = L.counters;
  a.queue = L.queue;
  a.claim = L.claim;
  a.pend = L.pend;
  a.log = L.log;
  a.log_cap = L.log_cap;
  a.log_n = L.log_n;
  a.log_fate = L.log_fate;
  a.digest = L.digest;
  a.rec = L.rec;
  a.rec_cap = L.rec_cap;
  a.rec_count = L.rec_count;
  a.mlp = L.mlp;
  a.chunk = L.chunk;
  a.sort_period = L.sort_period;
  a.n_lv = L.G_n_lv;
  dim3 grid(L.grid), block(kPool);
#define GNAV_LAUNCH(LOGV, CNTV, ORDV, PRECV) \
  hipLaunchKernelGGL((k_transport<LOGV, CNTV, ORDV, PRECV>), grid, block, 0, st, a)
#define GNAV_LAUNCH_ORDER(LOGV, CNTV)                                                    \
  do {                                                                                   \
    if (L.prec == kPrecScreened) GNAV_LAUNCH(LOGV, CNTV, kOrderPlain, kPrecScreened);    \
    else if (L.prec == kPrecPure) GNAV_LAUNCH(LOGV, CNTV, kOrderPlain, kPrecPure);       \
    else if (L.order == kOrderBound) GNAV_LAUNCH(LOGV, CNTV, kOrderBound, kPrecFP64);    \
    else if (L.order == kOrderLearned) GNAV_LAUNCH(LOGV, CNTV, kOrderLearned, kPrecFP64); \
    else GNAV_LAUNCH(LOGV, CNTV, kOrderPlain, kPrecFP64);                                \
  } while (0)
  if (L.log || L.digest) {
    if (L.count) GNAV_LAUNCH_ORDER(true, true);
    else GNAV_LAUNCH_ORDER(true, false);
  } else {
    if (L.count) GNAV_LAUNCH_ORDER(false, true);
    else GNAV_LAUNCH_ORDER(false, false);
  }
#undef GNAV_LAUNCH_ORDER
#undef GNAV_LAUNCH
  return hipGetLastError();
}

}  // namespace GNAV_POOL_NS

hipError_t GNAV_CAT(launch_transport_, GNAV_POOL_NS)(const TransportLaunch& L, hipStream_t st) {
  return GNAV_POOL_NS::launch(L, st);
}

}  // namespace gnav

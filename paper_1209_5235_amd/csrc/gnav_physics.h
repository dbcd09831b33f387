// gnav_physics.h -- device physics of the gamma loop (attenuation lookup,
// Compton sampling, direction rotation) and the transport kernel's
// argument block, shared by the transport and query translation units.
#pragma once

#include <hip/hip_runtime.h>

#include "gnav_device.h"
#include "gnav_internal.h"

namespace gnav {

// ---------------------------------------------------------------------------
// Transport
// ---------------------------------------------------------------------------

// Table position of energy E: node index i and weight w, linear in ln E
// over 257 nodes (clamped at both ends).
__device__ __forceinline__ void mu_index(const DevGeom& G, double E, int& i, double& w) {
  double x = (log(E) - G.lnE0) / G.dlnE;
  if (x < 0) i = 0;
  else if (x >= 255.0) i = 255;
  else i = (int)x;
  w = x - (double)i;
  w = dmin(dmax(w, 0.0), 1.0);
}

__device__ __forceinline__ void mu_parts(const DevGeom& G, int mat, int i, double w, double E, double& pe,
                                         double& co, double& pp) {
  const double* t = G.xs + (size_t)mat * 3 * kNNode;
  pe = (1.0 - w) * t[i] + w * t[i + 1];
  co = (1.0 - w) * t[kNNode + i] + w * t[kNNode + i + 1];
  pp = (1.0 - w) * t[2 * kNNode + i] + w * t[2 * kNNode + i + 1];
  if (E < 2.0 * kMe) pp = 0.0;
}

// Butcher-Messel sampling of the Klein-Nishina energy fraction eps = E'/E:
// a two-branch mixture (weights ln(1+2k) and (1-eps0^2)/2) with acceptance
// 1 - eps sin^2(theta) / (1 + eps^2); three draws per trial.
__device__ __forceinline__ void compton_sample(double E, Philox& rs, uint32_t s0, uint32_t s1, double& eps,
                                               double& onecost, double& sint2) {
  double k = E / kMe;
  double eps0 = 1.0 / (1.0 + 2.0 * k);
  double eps0sq = eps0 * eps0;
  double a1 = log(1.0 + 2.0 * k);
  double a2 = 0.5 * (1.0 - eps0sq);
  for (int trial = 0; trial < kMaxComptonTrials; trial++) {
    double r1 = rng_next(rs, s0, s1), r2 = rng_next(rs, s0, s1), r3 = rng_next(rs, s0, s1);
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

// Turn unit vector v by polar angle (cos, sin) and azimuth phi about itself.
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
  const int* geom_tbase;   // [geoms] first touchable (global) = the world
  int n_geoms;
  int n_events;
  uint32_t seed_lo, seed_hi;
  double ecut;
  int max_steps;
  double* edep_t;
  double* edep_ev;
  double* esc_ev;
  unsigned long long* counters;
  unsigned long long* queue;  // [0]: next primary
  const ClaimRec* claim;      // [n] the primaries in queue order, or null (the caller's order)
  double* pend;               // [lanes][6]: pending annihilation photon position and direction
  gnav_logrec* log;
  long log_cap;
  int* log_n;                 // [3 n] or null
  int* log_fate;              // [3 n] or null
  gnav_digest* digest;        // [3 n] per-track digests, or null
  gnav_crossing* rec;         // optional crossing recorder
  long rec_cap;
  unsigned long long* rec_count;
  MlpView mlp;                // candidate-ordering network (learned order)
  int chunk;                  // 0: each wave claims what it needs; > 0: the block claims chunks
  int sort_period;            // every sort_period-th round buckets the step phase by volume (0: never)
  int n_lv;                   // resident logical volumes (sort keys)
};

__device__ __forceinline__ void atomic_add_f64(double* p, double v) { unsafeAtomicAdd(p, v); }

}  // namespace gnav

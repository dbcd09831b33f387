// gnav_internal.h -- declarations shared by the host runtime and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "gnav.h"
#include "gnav_device.h"

namespace gnav {

// Energy classes of the claim order: half octaves from 1 keV, highest first;
// a batch over several geometries sorts by geometry, then energy class (at
// most kClaimMaxKeys keys: batches over more geometries keep their order).
constexpr int kClaimClasses = 64;
constexpr int kClaimMaxKeys = 1024;

// A primary copied into claim order, so that the transport reads the
// primaries it claims contiguously (72 bytes).
struct ClaimRec {
  double pos[3], dir[3], energy;
  int event, prim_id;
  int index;  // position in the caller's arrays (log and digest slots)
  int pad;
};
static_assert(sizeof(ClaimRec) == 72, "claim record layout");

// Device view of a candidate-ordering network (bf16 weights, float biases).
struct MlpView {
  const uint16_t* w1x;  // [128][6]
  const uint16_t* w1m;  // [n_class][128]
  const uint16_t* w2;   // [128][128]
  const uint16_t* w3;   // [64][128]
  const float* b1;
  const float* b2;
  const float* b3;
  int n_class;
};

struct TransportLaunch {
  DevGeom G;
  long n;
  ClaimRec* claim;         // [n] the primaries in queue order (decreasing energy), or null: as given
  unsigned* claim_cnt;     // [2 * claim_keys] key counts and cursors for building it
  int claim_keys;          // kClaimClasses, times the geometries for a batch with per-event geometries
  const int* event;
  const int* prim_id;
  const double* pos;
  const double* dir;
  const double* energy;
  const int* event_geom;
  int geom_default;
  const int* geom_tbase;
  int n_geoms;
  int n_events;
  uint64_t seed;
  double ecut;
  long max_steps;
  double* edep_t;
  double* edep_ev;
  double* esc_ev;
  unsigned long long* counters;
  unsigned long long* queue;
  double* pend;
  gnav_logrec* log;
  long log_cap;
  int* log_n;
  int* log_fate;
  gnav_digest* digest;
  int block;
  int grid;
  bool axis_boxes;  // every solid the batch can reach is a box placed without rotation
  bool spheres;     // some solid the batch can reach is a sphere section
  bool count;
  int order;
  int prec;  // kPrecFP64 / kPrecScreened / kPrecPure (FP32 forms use the plain order)
  int chunk;        // queue claim size per block (0: per wave, exactly what it needs)
  int sort_period;  // rounds between volume-bucketed step phases (0: never)
  int G_n_lv;       // resident logical volumes
  gnav_crossing* rec;
  long rec_cap;
  unsigned long long* rec_count;
  MlpView mlp;
};

bool mlp_view(const gnav_mlp* m, MlpView* out);
hipError_t launch_mlp_score(const MlpView& M, long n, const float* x, const int* cls, float* logits, int* pred,
                            hipStream_t st);
const gnav_ctx* mlp_owner(const gnav_mlp* m);
// Drop every binding of `mlp` in context c (the network is being freed).
void unbind_mlp(gnav_ctx* c, const gnav_mlp* mlp);

hipError_t launch_locate(const DevGeom& G, int W, int tbase, long n, const double* pos,
                         const double* dir, int* out, hipStream_t st);
// One ComputeStep query launch (gnav_compute_step_ex): n queries of one
// geometry whose world touchable is W (= tbase) with tcount touchables.
struct StepArgs {
  DevGeom G;
  int W, tbase, tcount;
  long n;
  const double* pos;
  const double* dir;
  const int* touch;         // per-geometry touchable ids, or null: locate first
  const double* max_step;   // or null
  double* step;
  int* lim;
  int* next;                // or null
  double* saf;              // or null
  double* normal;           // [n][3] or null
  int* normal_valid;        // or null
  MlpView mlp;              // order 2 only
};

hipError_t launch_step(const StepArgs& a, int prec, int order, hipStream_t st);
hipError_t launch_safety(const DevGeom& G, int W, int tbase, int tcount, long n, const double* pos,
                         const int* touch, double* out, int prec, hipStream_t st);
hipError_t launch_transport(const TransportLaunch& L, hipStream_t st);
// the transport kernel built for track pools of 64, 128 and 256 slots
hipError_t launch_transport_pool64(const TransportLaunch& L, hipStream_t st);
hipError_t launch_transport_pool64_axis_boxes(const TransportLaunch& L, hipStream_t st);
hipError_t launch_transport_pool64_spheres(const TransportLaunch& L, hipStream_t st);
hipError_t launch_transport_pool128_spheres(const TransportLaunch& L, hipStream_t st);
hipError_t launch_transport_pool256_spheres(const TransportLaunch& L, hipStream_t st);
hipError_t launch_transport_pool128(const TransportLaunch& L, hipStream_t st);
hipError_t launch_transport_pool256(const TransportLaunch& L, hipStream_t st);
hipError_t launch_free_path(const DevGeom& G, int W, long n, const double* pos, const double* dir,
                            const double* life, double E, double mu_mass, double* t_out, int* nb_out,
                            hipStream_t st);
// Zero `words` 8-byte words with a kernel (graph-capture safe, no memset node).
hipError_t launch_zero(void* p, size_t words, hipStream_t st);
// Zero up to four arrays of 8-byte words in one launch (null or empty ones skipped).
hipError_t launch_zero4(void* const p[4], const size_t words[4], hipStream_t st);

}  // namespace gnav

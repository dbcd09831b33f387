// gnav_device.h -- device-side geometry tables, solids and navigation for gfx950.
//
// Navigation answers the two questions of Sec. 3.2 (which volumes hold a
// point; where a ray next meets a boundary) on a placement hierarchy.  The
// paper's port kept a per-particle navigator with a stack of volumes and
// dispatched solid calls through "fork" functions (Sec. 3.3), and named
// register pressure from those structures as its GPU bottleneck (Sec. 5).
// Here a track's navigation state is a single touchable id (a placement path
// expanded on the host), every touchable carries its composed world->local
// transform, and solid dispatch is a switch over a type code read from
// structure-of-arrays tables.
//
// Solid rules (both entry points agree on surfaces): each solid is the
// intersection of components with signed values negative inside; d(p) is
// their maximum.  d < -tol/2 is inside, d > tol/2 outside, otherwise on the
// surface, where a direction counts as entering only if it points strictly
// inward through every face whose tolerance band holds the point.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include "gnav.h"

namespace gnav {

constexpr double kTol = 1e-9;
constexpr double kHalfTol = 0.5e-9;
constexpr double kInf = __builtin_inf();
constexpr double kMe = 0.51099895;  // electron rest energy, MeV (CODATA 2018)
constexpr double kTwoPi = 6.283185307179586;
constexpr int kNNode = 257;         // cross-section nodes, 1 keV .. 100 MeV
constexpr int kZeroPush = 10;
constexpr int kZeroKill = 25;
constexpr int kMaxComptonTrials = 1000;

enum : int { kBox = 0, kTubs = 1, kCons = 2, kOrb = 3, kTrd = 4, kSphere = 5 };
enum : int { kOut = -1, kIn = 1 };
enum : int { kLimMother = -1, kLimPE = -2, kLimCompton = -3, kLimPair = -4, kLimMaxStep = -5 };

// Solid info bits: type in the low nibble, then has_inner, has_phi.
constexpr int kInfoInner = 1 << 4;
constexpr int kInfoPhi = 1 << 5;

// Radial-solid parameter slots (12 doubles per solid).
enum : int { R_AO = 0, R_BO, R_CO, R_AI, R_BI, R_CI, R_DZ, R_NS0, R_NS1, R_NE0, R_NE1, kSolidPar = 12 };

// Touchable record: everything a step needs about the current volume except
// its transform, in one 16-byte load.
struct TRec {
  int lv;          // logical volume (global)
  int parent;      // parent touchable, -1 for a world
  int child_base;  // touchable of daughter slot 0
  int slot_kind;   // slot in the parent LV (low 16 bits) | transform kind << 16 | depth << 24
};

// Logical-volume record: solid, material, daughters and voxel grid together,
// so a mother's exit distance, safety and daughter search start from one
// record (256 bytes).
struct LRec {
  int info;        // solid type | kInfoInner | kInfoPhi
  int mat;
  int dau_base;    // first placement
  int dau_cnt;
  int vox;         // 1: voxel grid present
  int n[3];        // grid counts
  int node_base;
  int lclass;      // candidate-ordering class of a voxelised mother (-1: none)
  int wide;        // 1: its voxel nodes hold kOrderMinCand or more candidates on average
  int pad_i[5];
  double par[kSolidPar];  // solid parameters
  double vlo[3], vinv[3], vw[3];
  double pad_d[3];
};

// Placement record: mother->local transform (M = R^T row major, then t),
// the placed solid's bounding box in the mother frame, child LV and whether
// M is the identity (176 bytes).
struct PRec {
  double m[12];
  double box_lo[3], box_hi[3];  // placed solid's bounding box in the mother frame
  int lv;
  int kind;
  int pad[6];
};

// FP32 twin of a placement for the FP32-distance variant: the translation
// stays FP64 (the offset from the placement origin is formed in FP64 and
// then rounded, so local coordinates keep FP32's relative precision), the
// rotation, bounding box and the placed solid's parameters are float (160
// bytes, everything one candidate test reads).
struct PRecF {
  double t[3];
  float r[9];          // mother -> local rotation (R^T, row major)
  int kind;            // 0: no rotation
  float lo[3], hi[3];  // bounding box in the mother frame, rounded outward
  int info;            // solid info of the placed LV
  float par[kSolidPar];
  float bscale;        // largest |lo|, |hi| (rounding margin of the box test)
  float sscale;        // largest solid parameter magnitude (margin of the safety)
  float sgrow;         // 1 + largest cone slope |B| (margin growth with distance)
  int pad[2];
};

static_assert(sizeof(LRec) == 256, "LRec layout");
static_assert(sizeof(PRec) == 176, "PRec layout");
static_assert(sizeof(PRecF) == 160, "PRecF layout");

// All device tables, by value in kernel arguments.  Indices are global over
// every resident geometry.
struct DevGeom {
  const TRec* t;            // [T]
  const double* t_xf;       // [T][12] world->local: M (row major) then t
  const LRec* lv;           // [LV]
  const PRec* pv;           // [PV]
  const int2* vox_node;     // {candidate offset, count}
  const uint16_t* vox_cand; // daughter slots, ascending within a node
  const double* xs;         // [mat][3][257] attenuation, 1/mm
  const double* mat_rho;    // [mat] density, g/cm3
  const float4* pv_cyl;     // [PV] {rho min, rho max, z min, z max} of the placed solid about
                            //      the mother's z axis, rounded outward
  const PRecF* pvf;         // [PV] FP32 twins of the placements
  const float* lv_parf;     // [LV][12] FP32 twins of the LV solid parameters
  const int* nbr;           // [T][6] face neighbours of box touchables (global id, -1: none): the
                            //   touchable found just outside the centre of face 2 axis + (side > 0)
  double lnE0, dlnE;
};

// ---------------------------------------------------------------------------
// Small helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ double dmax(double a, double b) { return a > b ? a : b; }
__device__ __forceinline__ double dmin(double a, double b) { return a < b ? a : b; }

template <typename R>
struct Vec3 {
  R x, y, z;
};
using V3 = Vec3<double>;
using V3f = Vec3<float>;

__device__ __forceinline__ V3 xf_point(const double* __restrict__ m, int kind, V3 p) {
  double d0 = p.x - m[9], d1 = p.y - m[10], d2 = p.z - m[11];
#ifdef GNAV_AXIS_BOXES
  return V3{d0, d1, d2};  // every placement is a translation (see the solid dispatch)
#endif
  if (kind == 0) return V3{d0, d1, d2};
  return V3{m[0] * d0 + m[1] * d1 + m[2] * d2, m[3] * d0 + m[4] * d1 + m[5] * d2,
            m[6] * d0 + m[7] * d1 + m[8] * d2};
}

__device__ __forceinline__ V3 xf_dir(const double* __restrict__ m, int kind, V3 v) {
#ifdef GNAV_AXIS_BOXES
  return v;
#endif
  if (kind == 0) return v;
  return V3{m[0] * v.x + m[1] * v.y + m[2] * v.z, m[3] * v.x + m[4] * v.y + m[5] * v.z,
            m[6] * v.x + m[7] * v.y + m[8] * v.z};
}

// ---------------------------------------------------------------------------
// Solid functions, templated on the arithmetic type R.  The FP64 path
// instantiates them with double; the FP32-distance path (Sec. 5 names FP64
// throughput as a limit of the port) with float on coordinates local to the
// solid's centre.  Every constant is written as R(...) so the float
// instantiation carries no hidden double arithmetic.
// ---------------------------------------------------------------------------

// Half width of the surface band.  FP64 uses the navigation tolerance; the
// FP32 instantiation (used for steps only by the pure FP32 form) needs a
// band wider than FP32 rounding of coordinates of a few metres (2.4e-4 mm
// per unit in the last place at 3 m), so it uses 1e-3 mm.
constexpr float kHalfTolF = 1e-3f;
template <typename R>
__device__ __forceinline__ constexpr R half_tol();
template <>
__device__ __forceinline__ constexpr double half_tol<double>() { return kHalfTol; }
template <>
__device__ __forceinline__ constexpr float half_tol<float>() { return kHalfTolF; }

template <typename R>
__device__ __forceinline__ R tmax(R a, R b) { return a > b ? a : b; }
template <typename R>
__device__ __forceinline__ R tmin(R a, R b) { return a < b ? a : b; }

// ---------------------------------------------------------------------------
// Box (half lengths h)
// ---------------------------------------------------------------------------

template <typename R>
__device__ __forceinline__ R box_d(const R* h, Vec3<R> p) {
  return tmax(tmax(fabs(p.x) - h[0], fabs(p.y) - h[1]), fabs(p.z) - h[2]);
}

// Face of a box (half lengths h) nearest to the point q on or near its
// boundary: 2 axis + (q on the positive side), the axis of the largest
// |q_a| - h_a (the lowest axis on ties).
__device__ __forceinline__ int box_face(const double* h, V3 q) {
  const double sx = fabs(q.x) - h[0], sy = fabs(q.y) - h[1], sz = fabs(q.z) - h[2];
  int a = 0;
  double m = sx;
  double c = q.x;
  if (sy > m) {
    a = 1;
    m = sy;
    c = q.y;
  }
  if (sz > m) {
    a = 2;
    c = q.z;
  }
  return 2 * a + (c > 0 ? 1 : 0);
}

__device__ __forceinline__ int box_inside(const double* h, V3 p, bool has_v, V3 v) {
  double sx = fabs(p.x) - h[0], sy = fabs(p.y) - h[1], sz = fabs(p.z) - h[2];
  double d = dmax(dmax(sx, sy), sz);
  if (d < -kHalfTol) return kIn;
  if (d > kHalfTol) return kOut;
  if (!has_v) return kIn;
  if (fabs(sx) <= kHalfTol && p.x * v.x >= 0) return kOut;
  if (fabs(sy) <= kHalfTol && p.y * v.y >= 0) return kOut;
  if (fabs(sz) <= kHalfTol && p.z * v.z >= 0) return kOut;
  return kIn;
}

// Slab entry: the ray enters when it is inside all three slabs.
template <typename R>
__device__ __forceinline__ R box_dist_in(const R* h, Vec3<R> p, Vec3<R> v) {
  const R ht = half_tol<R>(), inf = R(kInf), zero = R(0);
  if (fabs(p.x) - h[0] >= -ht && p.x * v.x >= zero) return inf;
  if (fabs(p.y) - h[1] >= -ht && p.y * v.y >= zero) return inf;
  if (fabs(p.z) - h[2] >= -ht && p.z * v.z >= zero) return inf;
  R te = -inf, tx = inf;
  const R pc[3] = {p.x, p.y, p.z};
  const R vc[3] = {v.x, v.y, v.z};
#pragma unroll
  for (int i = 0; i < 3; i++) {
    if (vc[i] == zero) continue;
    R t1 = (-h[i] - pc[i]) / vc[i];
    R t2 = (h[i] - pc[i]) / vc[i];
    te = tmax(te, tmin(t1, t2));
    tx = tmin(tx, tmax(t1, t2));
  }
  if (te >= tx - ht) return inf;
  return te < ht ? zero : te;
}

template <typename R>
__device__ __forceinline__ R box_dist_out(const R* h, Vec3<R> p, Vec3<R> v) {
  const R ht = half_tol<R>(), zero = R(0);
  R t = R(kInf);
  const R pc[3] = {p.x, p.y, p.z};
  const R vc[3] = {v.x, v.y, v.z};
#pragma unroll
  for (int i = 0; i < 3; i++) {
    R sd;
    if (vc[i] > zero) sd = h[i] - pc[i];
    else if (vc[i] < zero) sd = h[i] + pc[i];
    else continue;
    if (sd <= ht) return zero;
    t = tmin(t, sd / fabs(vc[i]));
  }
  return t;
}

// ---------------------------------------------------------------------------
// Trapezoid: x and y half widths linear in z between -dz and +dz, a convex
// solid of six face planes +x, -x, +y, -y, +z, -z with unit outward normals
// (+-cx, 0, nzx), (0, +-cy, nzy), (0, 0, +-1) and offsets hx, hx, hy, hy, dz,
// dz, from q = {cx, nzx, hx, cy, nzy, hy, dz}.
// ---------------------------------------------------------------------------

template <typename R>
__device__ __forceinline__ R trd_plane(const R* q, int i, Vec3<R> p) {
  switch (i) {
    case 0: return (q[0] * p.x + q[1] * p.z) - q[2];
    case 1: return (-q[0] * p.x + q[1] * p.z) - q[2];
    case 2: return (q[3] * p.y + q[4] * p.z) - q[5];
    case 3: return (-q[3] * p.y + q[4] * p.z) - q[5];
    case 4: return p.z - q[6];
    default: return -p.z - q[6];
  }
}

template <typename R>
__device__ __forceinline__ R trd_dot(const R* q, int i, Vec3<R> v) {
  switch (i) {
    case 0: return q[0] * v.x + q[1] * v.z;
    case 1: return -q[0] * v.x + q[1] * v.z;
    case 2: return q[3] * v.y + q[4] * v.z;
    case 3: return -q[3] * v.y + q[4] * v.z;
    case 4: return v.z;
    default: return -v.z;
  }
}

template <typename R>
__device__ __forceinline__ R trd_d(const R* q, Vec3<R> p) {
  R d = trd_plane(q, 0, p);
#pragma unroll
  for (int i = 1; i < 6; i++) d = tmax(d, trd_plane(q, i, p));
  return d;
}

__device__ __forceinline__ int trd_inside(const double* q, V3 p, bool has_v, V3 v) {
  const double d = trd_d(q, p);
  if (d < -kHalfTol) return kIn;
  if (d > kHalfTol) return kOut;
  if (!has_v) return kIn;
#pragma unroll
  for (int i = 0; i < 6; i++)
    if (fabs(trd_plane(q, i, p)) <= kHalfTol && trd_dot(q, i, v) >= 0) return kOut;
  return kIn;
}

// Entry: the latest plane entry before the earliest plane exit; no entry
// through a face whose band holds p (or beyond it) that the ray does not
// cross inward; a start on the band moving in gives 0.
template <typename R>
__device__ __forceinline__ R trd_dist_in(const R* q, Vec3<R> p, Vec3<R> v) {
  const R ht = half_tol<R>(), inf = R(kInf), zero = R(0);
  R dp[6], dv[6];
#pragma unroll
  for (int i = 0; i < 6; i++) {
    dp[i] = trd_plane(q, i, p);
    dv[i] = trd_dot(q, i, v);
    if (dp[i] >= -ht && dv[i] >= zero) return inf;
  }
  R te = -inf, tx = inf;
#pragma unroll
  for (int i = 0; i < 6; i++) {
    if (dv[i] == zero) continue;
    const R t = -dp[i] / dv[i];
    if (dv[i] < zero) te = tmax(te, t);
    else tx = tmin(tx, t);
  }
  if (te >= tx - ht) return inf;
  return te < ht ? zero : te;
}

template <typename R>
__device__ __forceinline__ R trd_dist_out(const R* q, Vec3<R> p, Vec3<R> v) {
  const R ht = half_tol<R>(), zero = R(0);
  R t = R(kInf);
#pragma unroll
  for (int i = 0; i < 6; i++) {
    const R dv = trd_dot(q, i, v);
    if (!(dv > zero)) continue;
    const R sd = -trd_plane(q, i, p);
    if (sd <= ht) return zero;
    t = tmin(t, sd / dv);
  }
  return t;
}

// ---------------------------------------------------------------------------
// Orb (radius R)
// ---------------------------------------------------------------------------

template <typename R>
__device__ __forceinline__ R orb_d(R rad, Vec3<R> p) {
  return sqrt(p.x * p.x + p.y * p.y + p.z * p.z) - rad;
}

__device__ __forceinline__ int orb_inside(double rad, V3 p, bool has_v, V3 v) {
  double d = orb_d(rad, p);
  if (d < -kHalfTol) return kIn;
  if (d > kHalfTol) return kOut;
  if (!has_v) return kIn;
  return (p.x * v.x + p.y * v.y + p.z * v.z) < 0 ? kIn : kOut;
}

template <typename R>
__device__ __forceinline__ R orb_dist_in(R rad, Vec3<R> p, Vec3<R> v) {
  const R ht = half_tol<R>(), inf = R(kInf), zero = R(0);
  R rr = p.x * p.x + p.y * p.y + p.z * p.z;
  R sd = sqrt(rr) - rad;
  R b = p.x * v.x + p.y * v.y + p.z * v.z;
  if (sd < -ht) return zero;
  if (b >= zero) return inf;
  R c = rr - rad * rad;
  R disc = b * b - c;
  if (disc <= zero) return inf;
  R sq = sqrt(disc);
  R te = c / (sq - b);
  R tx = sq - b;
  if (te >= tx - ht) return inf;
  return te < ht ? zero : te;
}

template <typename R>
__device__ __forceinline__ R orb_dist_out(R rad, Vec3<R> p, Vec3<R> v) {
  const R ht = half_tol<R>(), zero = R(0);
  R rr = p.x * p.x + p.y * p.y + p.z * p.z;
  R sd = sqrt(rr) - rad;
  R b = p.x * v.x + p.y * v.y + p.z * v.z;
  if (sd >= -ht && b >= zero) return zero;
  R c = rr - rad * rad;
  R disc = b * b - c;
  if (disc < zero) disc = zero;
  R sq = sqrt(disc);
  R t = (b > zero) ? -c / (b + sq) : sq - b;
  return t > zero ? t : zero;
}

// ---------------------------------------------------------------------------
// Tube and cone sections: outer surface rho = Ao + Bo z, inner rho = Ai + Bi
// z (optional), slab |z| <= dz, phi wedge (optional, at most pi wide).
// ---------------------------------------------------------------------------

template <typename R>
struct RadComps {
  R ro, ri, z, pa, pb;
};

template <typename R>
__device__ __forceinline__ RadComps<R> rad_comps(const R* q, int info, Vec3<R> p) {
  const R inf = R(kInf);
  RadComps<R> k;
  R rho = sqrt(p.x * p.x + p.y * p.y);
  k.ro = (rho - (q[R_AO] + q[R_BO] * p.z)) * q[R_CO];
  k.ri = (info & kInfoInner) ? ((q[R_AI] + q[R_BI] * p.z) - rho) * q[R_CI] : -inf;
  k.z = fabs(p.z) - q[R_DZ];
  if (info & kInfoPhi) {
    k.pa = p.x * q[R_NS0] + p.y * q[R_NS1];
    k.pb = p.x * q[R_NE0] + p.y * q[R_NE1];
  } else {
    k.pa = -inf;
    k.pb = -inf;
  }
  return k;
}

template <typename R>
__device__ __forceinline__ R rad_dmax(const RadComps<R>& k) {
  return tmax(tmax(tmax(k.ro, k.ri), tmax(k.z, k.pa)), k.pb);
}

__device__ __forceinline__ int rad_inside(const double* q, int info, V3 p, bool has_v, V3 v) {
  RadComps<double> k = rad_comps(q, info, p);
  double d = rad_dmax(k);
  if (d < -kHalfTol) return kIn;
  if (d > kHalfTol) return kOut;
  if (!has_v) return kIn;
  double rho = sqrt(p.x * p.x + p.y * p.y);
  double rv = rho > 0 ? (p.x * v.x + p.y * v.y) / rho : 0.0;
  if (fabs(k.ro) <= kHalfTol && rv - q[R_BO] * v.z >= 0) return kOut;
  if ((info & kInfoInner) && fabs(k.ri) <= kHalfTol && -rv + q[R_BI] * v.z >= 0) return kOut;
  if (fabs(k.z) <= kHalfTol && p.z * v.z >= 0) return kOut;
  if (info & kInfoPhi) {
    if (fabs(k.pa) <= kHalfTol && v.x * q[R_NS0] + v.y * q[R_NS1] >= 0) return kOut;
    if (fabs(k.pb) <= kHalfTol && v.x * q[R_NE0] + v.y * q[R_NE1] >= 0) return kOut;
  }
  return kIn;
}

// Roots of f(t) = rho(t)^2 - (A + B z(t))^2 = a t^2 + 2 b t + c on the real
// sheet (A + B z >= 0); `want` selects the slope sign: +1 leaving rho <= R(z),
// -1 entering it.  Returns the smallest such root that is >= lo.
template <typename R>
__device__ __forceinline__ R radial_root(R A, R B, Vec3<R> p, Vec3<R> v, int want, R lo) {
  const R inf = R(kInf), zero = R(0);
  R R0 = A + B * p.z;
  R Rv = B * v.z;
  R a = v.x * v.x + v.y * v.y - Rv * Rv;
  R b = p.x * v.x + p.y * v.y - R0 * Rv;
  R c = p.x * p.x + p.y * p.y - R0 * R0;
  R t0, t1;
  int n;
  if (a == zero) {
    if (b == zero) return inf;
    t0 = -c / (R(2) * b);
    t1 = inf;
    n = 1;
  } else {
    R disc = b * b - a * c;
    if (disc < zero) return inf;
    R sq = sqrt(disc);
    R qq = (b >= zero) ? -(b + sq) : (sq - b);
    R r1 = qq / a;
    R r2 = (qq != zero) ? c / qq : r1;
    t0 = tmin(r1, r2);
    t1 = tmax(r1, r2);
    n = 2;
  }
  R best = inf;
  {
    R s = a * t0 + b;
    bool ok = want > 0 ? (s > zero) : (s < zero);
    if (ok && R0 + Rv * t0 >= zero && t0 >= lo) best = t0;
  }
  if (n == 2 && best == inf) {
    R s = a * t1 + b;
    bool ok = want > 0 ? (s > zero) : (s < zero);
    if (ok && R0 + Rv * t1 >= zero && t1 >= lo) best = t1;
  }
  return best;
}

template <typename R>
__device__ __forceinline__ bool rad_ok_except(const R* q, int info, Vec3<R> p, Vec3<R> v, R t, int skip) {
  const R ht = half_tol<R>();
  Vec3<R> r{p.x + t * v.x, p.y + t * v.y, p.z + t * v.z};
  RadComps<R> k = rad_comps(q, info, r);
  if (skip != 0 && k.ro > ht) return false;
  if (skip != 1 && k.ri > ht) return false;
  if (skip != 2 && k.z > ht) return false;
  if (skip != 3 && k.pa > ht) return false;
  if (skip != 4 && k.pb > ht) return false;
  return true;
}

// Entry distance, surface by surface: a crossing through one face counts if
// every other component holds at the crossing point.
template <typename R>
__device__ __forceinline__ R rad_dist_in(const R* q, int info, Vec3<R> p, Vec3<R> v) {
  const R ht = half_tol<R>(), inf = R(kInf), zero = R(0);
  RadComps<R> k = rad_comps(q, info, p);
  if (rad_dmax(k) < -ht) return zero;
  R rho = sqrt(p.x * p.x + p.y * p.y);
  R rv = rho > zero ? (p.x * v.x + p.y * v.y) / rho : zero;
  R best = inf;
  if (k.z >= -ht) {
    if (p.z * v.z >= zero) return inf;
    R t = k.z / fabs(v.z);
    if (t < zero) t = zero;
    if (rad_ok_except(q, info, p, v, t, 2)) best = tmin(best, t);
  }
  if (k.ro >= -ht) {
    if (rv - q[R_BO] * v.z >= zero) return inf;
    R t = radial_root(q[R_AO], q[R_BO], p, v, -1, -inf);
    if (t == inf) return inf;
    if (t < zero) t = zero;
    if (rad_ok_except(q, info, p, v, t, 0)) best = tmin(best, t);
  }
  if (info & kInfoInner) {
    R t = R(-1);
    if (fabs(k.ri) <= ht) {
      R vn = -rv + q[R_BI] * v.z;
      if (vn < zero) t = zero;
      else if (vn > zero) t = radial_root(q[R_AI], q[R_BI], p, v, +1, zero);
    } else {
      t = radial_root(q[R_AI], q[R_BI], p, v, +1, zero);
    }
    if (t >= zero && t < inf && rad_ok_except(q, info, p, v, t, 1)) best = tmin(best, t);
  }
  if (info & kInfoPhi) {
    if (k.pa >= -ht) {
      R dv = v.x * q[R_NS0] + v.y * q[R_NS1];
      if (dv >= zero) return inf;
      R t = k.pa / (-dv);
      if (t < zero) t = zero;
      if (rad_ok_except(q, info, p, v, t, 3)) best = tmin(best, t);
    }
    if (k.pb >= -ht) {
      R dv = v.x * q[R_NE0] + v.y * q[R_NE1];
      if (dv >= zero) return inf;
      R t = k.pb / (-dv);
      if (t < zero) t = zero;
      if (rad_ok_except(q, info, p, v, t, 4)) best = tmin(best, t);
    }
  }
  return best < ht ? zero : best;
}

template <typename R>
__device__ __forceinline__ R rad_dist_out(const R* q, int info, Vec3<R> p, Vec3<R> v) {
  const R ht = half_tol<R>(), zero = R(0);
  RadComps<R> k = rad_comps(q, info, p);
  R rho = sqrt(p.x * p.x + p.y * p.y);
  R rv = rho > zero ? (p.x * v.x + p.y * v.y) / rho : zero;
  R t = R(kInf);
  if (v.z != zero) {
    R sd = v.z > zero ? q[R_DZ] - p.z : q[R_DZ] + p.z;
    if (sd <= ht) return zero;
    t = tmin(t, sd / fabs(v.z));
  }
  if (k.ro >= -ht && rv - q[R_BO] * v.z >= zero) return zero;
  t = tmin(t, radial_root(q[R_AO], q[R_BO], p, v, +1, zero));
  if (info & kInfoInner) {
    if (k.ri >= -ht && -rv + q[R_BI] * v.z >= zero) return zero;
    t = tmin(t, radial_root(q[R_AI], q[R_BI], p, v, -1, zero));
  }
  if (info & kInfoPhi) {
    R dv = v.x * q[R_NS0] + v.y * q[R_NS1];
    if (k.pa >= -ht && dv >= zero) return zero;
    if (dv > zero) t = tmin(t, tmax(-k.pa / dv, zero));
    dv = v.x * q[R_NE0] + v.y * q[R_NE1];
    if (k.pb >= -ht && dv >= zero) return zero;
    if (dv > zero) t = tmin(t, tmax(-k.pb / dv, zero));
  }
  return t;
}

// ---------------------------------------------------------------------------
// Sphere sections: shell rmin <= r <= rmax, phi wedge (optional, at most pi
// wide), and up to two theta bounds, each the cone rho = B z (B = tan theta,
// perpendicular factor c = |cos theta|) whose inside (outer kind) or outside
// (inner kind) is kept, or for theta = pi/2 the half-space z <= 0 or z >= 0.
// q = {rmax, rmin, ns0, ns1, ne0, ne1, B1, c1, B2, c2}; the bound kinds sit in
// the solid info above the family bits.
// ---------------------------------------------------------------------------

enum : int { kTNone = 0, kTOuter = 1, kTInner = 2, kTZle = 3, kTZge = 4 };
constexpr int kInfoTheta = 6;  // bit offset of the first theta bound's kind (3 bits each)

__device__ __forceinline__ int sph_kind(int info, int j) { return (info >> (kInfoTheta + 3 * j)) & 7; }

template <typename R>
struct SphComps {
  R k[6];  // outer sphere, inner sphere, start phi, end phi, theta bound 1, theta bound 2
};

template <typename R>
__device__ __forceinline__ SphComps<R> sph_comps(const R* q, int info, Vec3<R> p) {
  const R inf = R(kInf);
  SphComps<R> c;
  const R r = sqrt(p.x * p.x + p.y * p.y + p.z * p.z);
  const R rho = sqrt(p.x * p.x + p.y * p.y);
  c.k[0] = r - q[0];
  c.k[1] = (info & kInfoInner) ? q[1] - r : -inf;
  if (info & kInfoPhi) {
    c.k[2] = p.x * q[2] + p.y * q[3];
    c.k[3] = p.x * q[4] + p.y * q[5];
  } else {
    c.k[2] = -inf;
    c.k[3] = -inf;
  }
#pragma unroll
  for (int j = 0; j < 2; j++) {
    const R B = q[6 + 2 * j], cc = q[7 + 2 * j];
    switch (sph_kind(info, j)) {
      case kTOuter: c.k[4 + j] = (rho - (R(0) + B * p.z)) * cc; break;
      case kTInner: c.k[4 + j] = ((R(0) + B * p.z) - rho) * cc; break;
      case kTZle: c.k[4 + j] = p.z; break;
      case kTZge: c.k[4 + j] = -p.z; break;
      default: c.k[4 + j] = -inf; break;
    }
  }
  return c;
}

template <typename R>
__device__ __forceinline__ R sph_dmax(const SphComps<R>& c) {
  R d = c.k[0];
#pragma unroll
  for (int i = 1; i < 6; i++) d = tmax(d, c.k[i]);
  return d;
}

// v . gradient of component i (unit gradients except that the cone's is
// scaled by 1 / c, which keeps its sign).
template <typename R>
__device__ __forceinline__ R sph_comp_dot(const R* q, int info, int i, Vec3<R> p, Vec3<R> v) {
  const R zero = R(0);
  const R r = sqrt(p.x * p.x + p.y * p.y + p.z * p.z);
  const R rho = sqrt(p.x * p.x + p.y * p.y);
  const R pv = p.x * v.x + p.y * v.y + p.z * v.z;
  const R rv = rho > zero ? (p.x * v.x + p.y * v.y) / rho : zero;
  switch (i) {
    case 0: return r > zero ? pv / r : zero;
    case 1: return r > zero ? -pv / r : zero;
    case 2: return v.x * q[2] + v.y * q[3];
    case 3: return v.x * q[4] + v.y * q[5];
    default: {
      const int j = i - 4;
      switch (sph_kind(info, j)) {
        case kTOuter: return rv - q[6 + 2 * j] * v.z;
        case kTInner: return -rv + q[6 + 2 * j] * v.z;
        case kTZle: return v.z;
        case kTZge: return -v.z;
        default: return zero;
      }
    }
  }
}

// The sphere section's inside test and distances are kept out of line: their
// six components would otherwise raise the register count of every kernel
// that dispatches over the solid families (the transport loop spills without
// this), while only steps in or at sphere sections pay for the call.
__device__ __attribute__((noinline)) int sph_inside(const double* q, int info, V3 p, bool has_v, V3 v) {
  const SphComps<double> c = sph_comps(q, info, p);
  const double d = sph_dmax(c);
  if (d < -kHalfTol) return kIn;
  if (d > kHalfTol) return kOut;
  if (!has_v) return kIn;
  bool out = false;
#pragma unroll
  for (int i = 0; i < 6; i++)
    if (c.k[i] > -kInf && fabs(c.k[i]) <= kHalfTol && sph_comp_dot(q, info, i, p, v) >= 0) out = true;
  return out ? kOut : kIn;
}

template <typename R>
__device__ __forceinline__ bool sph_ok_except(const R* q, int info, Vec3<R> p, Vec3<R> v, R t, int skip) {
  const R ht = half_tol<R>();
  const SphComps<R> c = sph_comps(q, info, Vec3<R>{p.x + t * v.x, p.y + t * v.y, p.z + t * v.z});
#pragma unroll
  for (int i = 0; i < 6; i++)
    if (i != skip && c.k[i] > ht) return false;
  return true;
}

// Entry, surface by surface as for tube and cone sections; the regions
// r <= rmax, the phi wedge, a cone's inside and a half-space are convex (no
// entry when the ray does not cross their face inward from its band or
// beyond), r >= rmin and a cone's outside are not.
template <typename R>
__device__ __attribute__((noinline)) R sph_dist_in(const R* q, int info, Vec3<R> p, Vec3<R> v) {
  const R ht = half_tol<R>(), inf = R(kInf), zero = R(0);
  const SphComps<R> c = sph_comps(q, info, p);
  if (sph_dmax(c) < -ht) return zero;
  const R rr = p.x * p.x + p.y * p.y + p.z * p.z;
  const R b = p.x * v.x + p.y * v.y + p.z * v.z;
  R best = inf;
  if (c.k[0] >= -ht) {
    if (b >= zero) return inf;
    const R cc = rr - q[0] * q[0];
    const R disc = b * b - cc;
    if (disc <= zero) return inf;
    const R sq = sqrt(disc);
    R t = cc / (sq - b);
    if (t < zero) t = zero;
    if (sph_ok_except(q, info, p, v, t, 0)) best = tmin(best, t);
  }
  if (info & kInfoInner) {
    R t = R(-1);
    const R cc = rr - q[1] * q[1];
    const R disc = b * b - cc;
    if (fabs(c.k[1]) <= ht) {
      if (b > zero) t = zero;
      else if (b < zero && disc > zero) t = sqrt(disc) - b;
    } else if (disc > zero) {
      const R sq = sqrt(disc);
      t = (b > zero) ? -cc / (b + sq) : sq - b;
    }
    if (t >= zero && t < inf && sph_ok_except(q, info, p, v, t, 1)) best = tmin(best, t);
  }
  if (info & kInfoPhi) {
#pragma unroll
    for (int j = 0; j < 2; j++) {
      const R dp = c.k[2 + j];
      if (dp >= -ht) {
        const R dv = v.x * q[2 + 2 * j] + v.y * q[3 + 2 * j];
        if (dv >= zero) return inf;
        R t = dp / (-dv);
        if (t < zero) t = zero;
        if (sph_ok_except(q, info, p, v, t, 2 + j)) best = tmin(best, t);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < 2; j++) {
    const int i = 4 + j;
    const int kind = sph_kind(info, j);
    if (kind == kTNone) continue;
    if (kind == kTOuter) {
      if (c.k[i] >= -ht) {
        if (sph_comp_dot(q, info, i, p, v) >= zero) return inf;
        R t = radial_root(zero, q[6 + 2 * j], p, v, -1, -inf);
        if (t == inf) return inf;
        if (t < zero) t = zero;
        if (sph_ok_except(q, info, p, v, t, i)) best = tmin(best, t);
      }
    } else if (kind == kTInner) {
      R t = R(-1);
      if (fabs(c.k[i]) <= ht) {
        const R vn = sph_comp_dot(q, info, i, p, v);
        if (vn < zero) t = zero;
        else if (vn > zero) t = radial_root(zero, q[6 + 2 * j], p, v, +1, zero);
      } else {
        t = radial_root(zero, q[6 + 2 * j], p, v, +1, zero);
      }
      if (t >= zero && t < inf && sph_ok_except(q, info, p, v, t, i)) best = tmin(best, t);
    } else {
      if (c.k[i] >= -ht) {
        const R vn = kind == kTZle ? v.z : -v.z;
        if (vn >= zero) return inf;
        R t = c.k[i] / (-vn);
        if (t < zero) t = zero;
        if (sph_ok_except(q, info, p, v, t, i)) best = tmin(best, t);
      }
    }
  }
  return best < ht ? zero : best;
}

template <typename R>
__device__ __attribute__((noinline)) R sph_dist_out(const R* q, int info, Vec3<R> p, Vec3<R> v) {
  const R ht = half_tol<R>(), zero = R(0);
  const SphComps<R> c = sph_comps(q, info, p);
  const R rr = p.x * p.x + p.y * p.y + p.z * p.z;
  const R b = p.x * v.x + p.y * v.y + p.z * v.z;
  R t = R(kInf);
  if (c.k[0] >= -ht && b >= zero) return zero;
  {
    const R cc = rr - q[0] * q[0];
    R disc = b * b - cc;
    if (disc < zero) disc = zero;
    const R sq = sqrt(disc);
    const R to = (b > zero) ? -cc / (b + sq) : sq - b;
    t = tmin(t, to > zero ? to : zero);
  }
  if (info & kInfoInner) {
    if (c.k[1] >= -ht && b <= zero) return zero;
    if (b < zero) {
      const R cc = rr - q[1] * q[1];
      const R disc = b * b - cc;
      if (disc > zero) {
        const R ti = cc / (sqrt(disc) - b);
        t = tmin(t, ti > zero ? ti : zero);
      }
    }
  }
  if (info & kInfoPhi) {
#pragma unroll
    for (int j = 0; j < 2; j++) {
      const R dp = c.k[2 + j];
      const R dv = v.x * q[2 + 2 * j] + v.y * q[3 + 2 * j];
      if (dp >= -ht && dv >= zero) return zero;
      if (dv > zero) {
        R tp = -dp / dv;
        if (tp < zero) tp = zero;
        t = tmin(t, tp);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < 2; j++) {
    const int i = 4 + j;
    const int kind = sph_kind(info, j);
    if (kind == kTNone) continue;
    const R vn = sph_comp_dot(q, info, i, p, v);
    if (c.k[i] >= -ht && vn >= zero) return zero;
    if (kind == kTOuter) {
      t = tmin(t, radial_root(zero, q[6 + 2 * j], p, v, +1, zero));
    } else if (kind == kTInner) {
      t = tmin(t, radial_root(zero, q[6 + 2 * j], p, v, -1, zero));
    } else if (vn > zero) {
      const R sd = -c.k[i];
      if (sd <= ht) return zero;
      t = tmin(t, sd / vn);
    }
  }
  return t;
}

// ---------------------------------------------------------------------------
// Surface normal (Sec. 3.2 asks for the normal of the boundary surface at the
// crossing point).  A solid's signed value is the largest of its components,
// so at a surface point its outward normal is the gradient of the largest
// component (the lowest component on ties); components within the tolerance
// of that largest value also hold the point, and two or more of them mean an
// edge or a corner.  Returns that count and writes the unit normal in the
// solid's frame.
// ---------------------------------------------------------------------------

__device__ __forceinline__ int solid_normal(int info, const double* q, V3 p, V3& n) {
#ifndef GNAV_AXIS_BOXES
  if ((info & 15) == kTrd) {
    double c[6];
#pragma unroll
    for (int i = 0; i < 6; i++) c[i] = trd_plane(q, i, p);
    int m = 0;
#pragma unroll
    for (int i = 1; i < 6; i++)
      if (c[i] > c[m]) m = i;
    int faces = 0;
#pragma unroll
    for (int i = 0; i < 6; i++)
      if (c[i] >= c[m] - kTol) faces++;
    switch (m) {
      case 0: n = V3{q[0], 0.0, q[1]}; break;
      case 1: n = V3{-q[0], 0.0, q[1]}; break;
      case 2: n = V3{0.0, q[3], q[4]}; break;
      case 3: n = V3{0.0, -q[3], q[4]}; break;
      case 4: n = V3{0.0, 0.0, 1.0}; break;
      default: n = V3{0.0, 0.0, -1.0}; break;
    }
    return faces;
  }
#ifdef GNAV_SPHERES
  if ((info & 15) == kSphere) {
    const SphComps<double> c = sph_comps(q, info, p);
    int m = 0;
    double km = c.k[0];
#pragma unroll
    for (int i = 1; i < 6; i++)
      if (c.k[i] > km) {
        m = i;
        km = c.k[i];
      }
    int faces = 0;
#pragma unroll
    for (int i = 0; i < 6; i++)
      if (c.k[i] >= km - kTol) faces++;
    const double r = sqrt(p.x * p.x + p.y * p.y + p.z * p.z);
    const double rho = sqrt(p.x * p.x + p.y * p.y);
    const double ex = rho > 0 ? p.x / rho : 1.0, ey = rho > 0 ? p.y / rho : 0.0;
    const V3 u = r > 0 ? V3{p.x / r, p.y / r, p.z / r} : V3{0.0, 0.0, 1.0};
    switch (m) {
      case 0: n = u; break;
      case 1: n = V3{-u.x, -u.y, -u.z}; break;
      case 2: n = V3{q[2], q[3], 0.0}; break;
      case 3: n = V3{q[4], q[5], 0.0}; break;
      default: {
        const int j = m - 4;
        const double B = q[6 + 2 * j], cc = q[7 + 2 * j];
        switch (sph_kind(info, j)) {
          case kTOuter: n = V3{cc * ex, cc * ey, -cc * B}; break;
          case kTInner: n = V3{-cc * ex, -cc * ey, cc * B}; break;
          case kTZle: n = V3{0.0, 0.0, 1.0}; break;
          default: n = V3{0.0, 0.0, -1.0}; break;
        }
      }
    }
    return faces;
  }
#endif
  if ((info & 15) == kOrb) {
    const double r = sqrt(p.x * p.x + p.y * p.y + p.z * p.z);
    n = r > 0 ? V3{p.x / r, p.y / r, p.z / r} : V3{0.0, 0.0, 1.0};
    return 1;
  }
  if ((info & 15) != kBox) {
    const RadComps<double> k = rad_comps(q, info, p);
    const double c[5] = {k.ro, k.ri, k.z, k.pa, k.pb};
    int m = 0;
#pragma unroll
    for (int i = 1; i < 5; i++)
      if (c[i] > c[m]) m = i;
    int faces = 0;
#pragma unroll
    for (int i = 0; i < 5; i++)
      if (c[i] >= c[m] - kTol) faces++;
    const double rho = sqrt(p.x * p.x + p.y * p.y);
    const double ux = rho > 0 ? p.x / rho : 1.0, uy = rho > 0 ? p.y / rho : 0.0;
    switch (m) {
      case 0: n = V3{ux * q[R_CO], uy * q[R_CO], -q[R_BO] * q[R_CO]}; break;
      case 1: n = V3{-ux * q[R_CI], -uy * q[R_CI], q[R_BI] * q[R_CI]}; break;
      case 2: n = V3{0.0, 0.0, p.z < 0 ? -1.0 : 1.0}; break;
      case 3: n = V3{q[R_NS0], q[R_NS1], 0.0}; break;
      default: n = V3{q[R_NE0], q[R_NE1], 0.0}; break;
    }
    return faces;
  }
#endif
  const double c[3] = {fabs(p.x) - q[0], fabs(p.y) - q[1], fabs(p.z) - q[2]};
  int m = 0;
  if (c[1] > c[m]) m = 1;
  if (c[2] > c[m]) m = 2;
  int faces = 0;
#pragma unroll
  for (int i = 0; i < 3; i++)
    if (c[i] >= c[m] - kTol) faces++;
  const double pc[3] = {p.x, p.y, p.z};
  const double sg = pc[m] < 0 ? -1.0 : 1.0;
  n = V3{m == 0 ? sg : 0.0, m == 1 ? sg : 0.0, m == 2 ? sg : 0.0};
  return faces;
}

// ---------------------------------------------------------------------------
// Dispatch over solid families ("fork" by type code)
//
// Sphere sections are dispatched only in translation units built with
// GNAV_SPHERES (the query kernels always; the transport kernel in builds of
// its own that the host launches when a batch can reach a sphere section):
// their code would otherwise cost every other geometry registers.
//
// A translation unit built with GNAV_AXIS_BOXES compiles the box code alone
// and treats every placement as a translation (the point and direction maps
// above): the host launches that build of the transport kernel only when
// every solid of the geometries a batch can reach is a box placed without
// rotation, and then it gives the same results with fewer registers and
// branches.  Device code is compiled per translation unit (no device
// linking), so the two forms never meet.
// ---------------------------------------------------------------------------

__device__ __forceinline__ int solid_inside(int info, const double* q, V3 p, bool has_v, V3 v) {
#ifdef GNAV_AXIS_BOXES
  return box_inside(q, p, has_v, v);
#else
  switch (info & 15) {
    case kBox: return box_inside(q, p, has_v, v);
    case kOrb: return orb_inside(q[0], p, has_v, v);
    case kTrd: return trd_inside(q, p, has_v, v);
#ifdef GNAV_SPHERES
    case kSphere: return sph_inside(q, info, p, has_v, v);
#endif
    default: return rad_inside(q, info, p, has_v, v);
  }
#endif
}

template <typename R>
__device__ __forceinline__ R solid_d(int info, const R* q, Vec3<R> p) {
#ifdef GNAV_AXIS_BOXES
  return box_d(q, p);
#else
  switch (info & 15) {
    case kBox: return box_d(q, p);
    case kOrb: return orb_d(q[0], p);
    case kTrd: return trd_d(q, p);
#ifdef GNAV_SPHERES
    case kSphere: return sph_dmax(sph_comps(q, info, p));
#endif
    default: return rad_dmax(rad_comps(q, info, p));
  }
#endif
}

template <typename R>
__device__ __forceinline__ R solid_dist_in(int info, const R* q, Vec3<R> p, Vec3<R> v) {
#ifdef GNAV_AXIS_BOXES
  return box_dist_in(q, p, v);
#else
  switch (info & 15) {
    case kBox: return box_dist_in(q, p, v);
    case kOrb: return orb_dist_in(q[0], p, v);
    case kTrd: return trd_dist_in(q, p, v);
#ifdef GNAV_SPHERES
    case kSphere: return sph_dist_in(q, info, p, v);
#endif
    default: return rad_dist_in(q, info, p, v);
  }
#endif
}

template <typename R>
__device__ __forceinline__ R solid_dist_out(int info, const R* q, Vec3<R> p, Vec3<R> v) {
#ifdef GNAV_AXIS_BOXES
  return box_dist_out(q, p, v);
#else
  switch (info & 15) {
    case kBox: return box_dist_out(q, p, v);
    case kOrb: return orb_dist_out(q[0], p, v);
    case kTrd: return trd_dist_out(q, p, v);
#ifdef GNAV_SPHERES
    case kSphere: return sph_dist_out(q, info, p, v);
#endif
    default: return rad_dist_out(q, info, p, v);
  }
#endif
}

// ---------------------------------------------------------------------------
// Voxel grids: a uniform grid per mother LV over its extent; each node lists
// the daughters whose padded bounding box meets the node, in slot order.
// ---------------------------------------------------------------------------

__device__ __forceinline__ int vox_axis_index(double p, double lo, double inv_w, int n) {
  double x = (p - lo) * inv_w;
  x = dmin(dmax(x, 0.0), (double)(n - 1));
  return (int)x;
}

// Work counters for the roofline accounting, by solid family (the low two
// bits of the solid info: box, tubs, cons, orb); compiled out when not
// wanted.  `frames` counts frame maps: one per daughter candidate examined
// (its entry distance, safety and inside test share one) and one per
// placement level of every touchable frame.
template <bool ON>
struct NavCount {
  static constexpr int F = GNAV_NFAMILIES;
  unsigned din[F] = {}, dout[F] = {}, dsaf[F] = {}, dins[F] = {};
  unsigned frames = 0, nodes = 0, dist_in32 = 0;
  __device__ __forceinline__ static void bump(unsigned (&a)[F], int info) {
    const int t = info & 15;
#pragma unroll
    for (int f = 0; f < F; f++) a[f] += t == f;
  }
  // daughter entry distance (FP64 or FP32), with its candidate frame unless
  // that was counted with the candidate's safety
  __device__ __forceinline__ void in(int info, bool own_frame = true) {
    if (ON) {
      bump(din, info);
      frames += own_frame ? 1u : 0u;
    }
  }
  __device__ __forceinline__ void in32(int info) {
    if (ON) {
      bump(din, info);
      frames++;
      dist_in32++;
    }
  }
  // mother exit distance
  __device__ __forceinline__ void out(int info) { if (ON) bump(dout, info); }
  // isotropic distance (safety); own_frame: a candidate examined for its safety alone
  __device__ __forceinline__ void saf(int info, bool own_frame) {
    if (ON) {
      bump(dsaf, info);
      frames += own_frame ? 1u : 0u;
    }
  }
  // point-in-solid test; own_frame: a daughter candidate's
  __device__ __forceinline__ void ins(int info, bool own_frame) {
    if (ON) {
      bump(dins, info);
      frames += own_frame ? 1u : 0u;
    }
  }
  __device__ __forceinline__ void levels(int n) { if (ON) frames += (unsigned)n; }
  __device__ __forceinline__ void node() { if (ON) nodes++; }
  __device__ __forceinline__ unsigned total(const unsigned (&a)[F]) const {
    unsigned s = 0;
#pragma unroll
    for (int f = 0; f < F; f++) s += a[f];
    return s;
  }
};

template <bool C>
__device__ __forceinline__ bool daughter_holds(const DevGeom& G, int pv, V3 pl, bool has_v, V3 vl,
                                               NavCount<C>& nc) {
  const PRec& P = G.pv[pv];
  int kind = P.kind;
  V3 pd = xf_point(P.m, kind, pl);
  V3 vd = xf_dir(P.m, kind, vl);
  const LRec& L = G.lv[P.lv];
  nc.ins(L.info, true);
  return solid_inside(L.info, L.par, pd, has_v, vd) == kIn;
}

// Daughter slot of mother record L holding (pl, vl): first match in slot order.
template <bool C>
__device__ __forceinline__ int find_daughter(const DevGeom& G, const LRec& L, V3 pl, bool has_v, V3 vl,
                                             int blocked, NavCount<C>& nc) {
  int cnt = L.dau_cnt;
  if (cnt == 0) return -1;
  int base = L.dau_base;
  if (!L.vox) {
    for (int k = 0; k < cnt; k++) {
      if (k == blocked) continue;
      if (daughter_holds(G, base + k, pl, has_v, vl, nc)) return k;
    }
    return -1;
  }
  int ix = vox_axis_index(pl.x, L.vlo[0], L.vinv[0], L.n[0]);
  int iy = vox_axis_index(pl.y, L.vlo[1], L.vinv[1], L.n[1]);
  int iz = vox_axis_index(pl.z, L.vlo[2], L.vinv[2], L.n[2]);
  int2 nd = G.vox_node[L.node_base + (ix * L.n[1] + iy) * L.n[2] + iz];
  for (int c = 0; c < nd.y; c++) {
    int k = G.vox_cand[nd.x + c];
    if (k == blocked) continue;
    if (daughter_holds(G, base + k, pl, has_v, vl, nc)) return k;
  }
  return -1;
}

__device__ __forceinline__ int trec_kind(const TRec& r) { return (r.slot_kind >> 16) & 0xFF; }
__device__ __forceinline__ int trec_depth(const TRec& r) { return (int)((unsigned)r.slot_kind >> 24); }
__device__ __forceinline__ int trec_slot(const TRec& r) { return r.slot_kind & 0xFFFF; }

// Descend from touchable T (holding the point, given in T's frame).  Also
// reports the LV of the touchable found and its transform kind, packed as
// (lv << 1) | kind.
template <bool C>
__device__ __forceinline__ int descend_local(const DevGeom& G, int T, V3 pl, bool has_v, V3 vl, int blocked,
                                             NavCount<C>& nc, int* lv_out = nullptr) {
  for (;;) {
    TRec tr = G.t[T];
    const LRec& L = G.lv[tr.lv];
    int k = find_daughter(G, L, pl, has_v, vl, blocked, nc);
    if (k < 0) {
      if (lv_out) *lv_out = (tr.lv << 1) | trec_kind(tr);
      return T;
    }
    const PRec& P = G.pv[L.dau_base + k];
    int pk = P.kind;
    pl = xf_point(P.m, pk, pl);
    vl = xf_dir(P.m, pk, vl);
    nc.levels(1);
    T = tr.child_base + k;
    blocked = -1;
  }
}

__device__ __forceinline__ void touchable_frame(const DevGeom& G, int T, int kind, V3 pg, V3 vg, V3& pl,
                                                V3& vl) {
  const double* m = G.t_xf + (size_t)T * 12;
  pl = xf_point(m, kind, pg);
  vl = xf_dir(m, kind, vg);
}

template <bool C>
__device__ __forceinline__ int descend(const DevGeom& G, int T, V3 pg, bool has_v, V3 vg, int blocked,
                                       NavCount<C>& nc) {
  V3 pl, vl;
  const TRec tr = G.t[T];
  touchable_frame(G, T, trec_kind(tr), pg, vg, pl, vl);
  nc.levels(trec_depth(tr));
  return descend_local(G, T, pl, has_v, vl, blocked, nc);
}

// LocateGlobalPoint from the world touchable W.
template <bool C>
__device__ __forceinline__ int locate(const DevGeom& G, int W, V3 pg, bool has_v, V3 vg, NavCount<C>& nc) {
  const LRec& L = G.lv[G.t[W].lv];
  nc.ins(L.info, false);
  if (solid_inside(L.info, L.par, pg, has_v, vg) == kOut) return -1;
  return descend_local(G, W, pg, has_v, vg, -1, nc);
}

// Relocation after a geometry step: enter daughter `lim`, or climb out of
// the volume(s) left and search the parent with the left volume excluded.
template <bool C>
__device__ __forceinline__ int relocate(const DevGeom& G, int T, const TRec& tr, V3 pg, V3 vg, int lim,
                                        NavCount<C>& nc) {
  if (lim >= 0) return descend(G, tr.child_base + lim, pg, true, vg, -1, nc);
  int left_slot = trec_slot(tr);
  int P = tr.parent;
  while (P >= 0) {
    TRec pr = G.t[P];
    V3 pl, vl;
    touchable_frame(G, P, trec_kind(pr), pg, vg, pl, vl);
    nc.levels(trec_depth(pr));
    const LRec& L = G.lv[pr.lv];
    nc.ins(L.info, false);
    if (solid_inside(L.info, L.par, pl, true, vl) != kOut)
      return descend_local(G, P, pl, true, vl, left_slot, nc);
    left_slot = trec_slot(pr);
    P = pr.parent;
  }
  return -1;
}

// One navigation fix-up shared by every way a track reaches a new position:
// starting (locate from the world touchable T), entering daughter `lim` of
// T, or leaving T (climb while outside the parent, then search it with the
// left volume excluded).  Returns the new touchable (-1: outside the world)
// and (its LV << 1) | transform kind.
//
// Leaving a box through face `face` (0-5, -1 unknown) first tries that face's
// neighbour N from G.nbr (never an ancestor of the box): when N holds the
// point (the same inside test with the direction rule), the answer is the
// descent from N, which is what the climb and search reach.  In a geometry of
// non-overlapping volumes the touchables other than the box left that hold a
// point under the direction rule form one chain from the world (siblings
// sharing a face are told apart by the sign of v.n), so the climb stops at
// the lowest common ancestor of the box and N, whose search (the box's branch
// excluded) enters N's branch, and the descent below N is the same.
// Otherwise the climb and search run as usual.
enum : int { kNavStart = 1, kNavEnter = 2, kNavExit = 3 };

template <bool C>
__device__ __forceinline__ int navigate(const DevGeom& G, int mode, int T, int lim, V3 x, V3 v, int& lvk_out,
                                        NavCount<C>& nc, int face = -1) {
  int cur = -1, blocked = -1;
  V3 pl = x, vl = v;
  if (mode == kNavExit && face >= 0) {
    const int N = G.nbr[(long)T * 6 + face];
    if (N >= 0) {
      const TRec tn = G.t[N];
      touchable_frame(G, N, trec_kind(tn), x, v, pl, vl);
      nc.levels(trec_depth(tn));
      const LRec& L = G.lv[tn.lv];
      nc.ins(L.info, false);
      if (solid_inside(L.info, L.par, pl, true, vl) == kIn) return descend_local(G, N, pl, true, vl, -1, nc, &lvk_out);
    }
  }
  if (mode == kNavStart) {
    const LRec& L = G.lv[G.t[T].lv];
    nc.ins(L.info, false);
    if (solid_inside(L.info, L.par, x, true, v) != kOut) cur = T;  // world frame = global frame
  } else if (mode == kNavEnter) {
    cur = G.t[T].child_base + lim;
    const TRec tc = G.t[cur];
    touchable_frame(G, cur, trec_kind(tc), x, v, pl, vl);
    nc.levels(trec_depth(tc));
  } else {
    TRec tr = G.t[T];
    int left_slot = trec_slot(tr);
    int P = tr.parent;
    while (P >= 0) {
      TRec pr = G.t[P];
      touchable_frame(G, P, trec_kind(pr), x, v, pl, vl);
      nc.levels(trec_depth(pr));
      const LRec& L = G.lv[pr.lv];
      nc.ins(L.info, false);
      if (solid_inside(L.info, L.par, pl, true, vl) != kOut) {
        cur = P;
        blocked = left_slot;
        break;
      }
      left_slot = trec_slot(pr);
      P = pr.parent;
    }
  }
  if (cur < 0) return -1;
  return descend_local(G, cur, pl, true, vl, blocked, nc, &lvk_out);
}

// Entry distance and safety of daughter placement pv, mother frame (pl, vl).
// `own_frame`: the candidate is examined for its safety alone (its frame is
// not already counted with an entry distance).
template <bool C>
__device__ __forceinline__ double daughter_dist_in(const DevGeom& G, int pv, V3 pl, V3 vl, NavCount<C>& nc,
                                                   bool own_frame = true) {
  const PRec& P = G.pv[pv];
  int kind = P.kind;
  V3 pd = xf_point(P.m, kind, pl);
  V3 vd = xf_dir(P.m, kind, vl);
  const LRec& L = G.lv[P.lv];
  nc.in(L.info, own_frame);
  return solid_dist_in(L.info, L.par, pd, vd);
}

template <bool C>
__device__ __forceinline__ double daughter_safety_in(const DevGeom& G, int pv, V3 pl, NavCount<C>& nc,
                                                     bool own_frame = false) {
  const PRec& P = G.pv[pv];
  V3 pd = xf_point(P.m, P.kind, pl);
  const LRec& L = G.lv[P.lv];
  nc.saf(L.info, own_frame);
  double d = solid_d(L.info, L.par, pd);
  return d > 0 ? d : 0.0;
}

// Lower bound on the entry distance of placement pv from (pl, vl) in the
// mother frame: the larger of the ray's entry into the placed bounding box
// (+inf on a miss) and the daughter's isotropic safety.  `saf` receives the
// safety alone.
__device__ __forceinline__ double daughter_lower_bound(const DevGeom& G, int pv, V3 pl, V3 vl, double& saf) {
  const PRec& P = G.pv[pv];
  const double pc[3] = {pl.x, pl.y, pl.z};
  const double vc[3] = {vl.x, vl.y, vl.z};
  double te = 0.0, tx = kInf;
#pragma unroll
  for (int a = 0; a < 3; a++) {
    double lo = P.box_lo[a], hi = P.box_hi[a];
    if (vc[a] == 0.0) {
      if (pc[a] < lo || pc[a] > hi) tx = -1.0;
      continue;
    }
    double t1 = (lo - pc[a]) / vc[a], t2 = (hi - pc[a]) / vc[a];
    te = dmax(te, dmin(t1, t2));
    tx = dmin(tx, dmax(t1, t2));
  }
  V3 pd = xf_point(P.m, P.kind, pl);
  const LRec& L = G.lv[P.lv];
  double d = solid_d(L.info, L.par, pd);
  saf = d > 0 ? d : 0.0;
  if (te > tx) return kInf;
  return dmax(te, saf);
}

// True when the ray (pl, vl) certainly meets placement P's bounding box
// beyond distance s or not at all (parallel outside a slab, or the box behind
// it on an axis): the bounding-box half of daughter_lower_bound(...)
// (1 - 1e-12) - kTol > s, written with products instead of quotients.  A ray
// that misses the box obliquely is not caught (the caller then evaluates the
// candidate exactly).
__device__ __forceinline__ bool box_beyond(const PRec& P, V3 pl, V3 vl, double s) {
  const double pc[3] = {pl.x, pl.y, pl.z};
  const double vc[3] = {vl.x, vl.y, vl.z};
  const double reach = s + kTol;
#pragma unroll
  for (int a = 0; a < 3; a++) {
    const double lo = P.box_lo[a], hi = P.box_hi[a];
    if (vc[a] > 0.0) {
      if (hi < pc[a]) return true;
      if ((lo - pc[a]) * (1.0 - 1e-12) > reach * vc[a]) return true;
    } else if (vc[a] < 0.0) {
      if (lo > pc[a]) return true;
      if ((pc[a] - hi) * (1.0 - 1e-12) > reach * -vc[a]) return true;
    } else if (pc[a] < lo || pc[a] > hi) {
      return true;
    }
  }
  return false;
}

// Isotropic lower bound on the distance from a point (rho = its distance to
// the mother's z axis, z) to a placed solid, from the solid's enclosing
// annular cylinder c = {rho min, rho max, z min, z max}: a point outside the
// radial band is at least the radial gap away from every point of it, and
// likewise along z.  16 bytes per candidate, no placement or solid record.
__device__ __forceinline__ double cyl_bound(float4 c, double rho, double z) {
  const double dr = dmax((double)c.x - rho, rho - (double)c.y);
  const double dz = dmax((double)c.z - z, z - (double)c.w);
  return dmax(dmax(dr, dz), 0.0);
}

// Candidate orders for the start node of a step walk.  Nodes with fewer
// candidates than kOrderMinCand are walked in slot order (with two, an
// ordering pass costs more than it can save), and so are all nodes of mothers
// whose nodes hold fewer than kOrderMinCand candidates on average (LRec.wide
// unset): there the ordering pass costs more than its rare skips save.
enum : int { kOrderPlain = 0, kOrderBound = 1, kOrderLearned = 2 };
constexpr int kOrderMinCand = 3;
// FP32 screening ranks every candidate of a node by its FP32 entry distance
// before the FP64 evaluations; a candidate's FP32 distance costs about what
// its FP64 one does (both wait on the same placement and solid records), so
// nodes with fewer than kScreenMinCand candidates are walked in FP64.
constexpr int kScreenMinCand = 6;

// ComputeStep in the mother frame (pl, vl) of a touchable with LV record L:
// the mother's exit distance against daughter entry distances, collected by
// walking the voxel nodes along the ray until the best distance lies strictly
// inside the current node.  The mother wins ties, then the lowest slot.
// Also returns the voxel-limited safety at the start point and the start
// node {candidate offset, count} (count 0 without voxels).
//
// ORDER changes only the order in which the start node's candidates are
// examined, never the result: the bound order evaluates the candidate with
// the smallest lower bound first, the learned order the candidate position
// `pred`; the others are then evaluated only when their lower bound (with a
// rounding margin) does not exceed the best distance so far, so a skipped
// candidate can neither beat nor tie it.
template <bool C, int ORDER = kOrderPlain>
__device__ __forceinline__ double compute_step(const DevGeom& G, const LRec& L, V3 pl, V3 vl, int& lim,
                                               double& safety, NavCount<C>& nc, int pred = -1,
                                               int2* start_node = nullptr) {
  const int info = L.info;
  double s = solid_dist_out(info, L.par, pl, vl);
  double md = solid_d(info, L.par, pl);
  double saf = md < 0 ? -md : 0.0;
  nc.out(info);
  nc.saf(info, false);
  lim = kLimMother;
  if (start_node) *start_node = int2{0, 0};
  int cnt = L.dau_cnt;
  if (cnt == 0) {
    safety = saf;
    return s;
  }
  int base = L.dau_base;
  if (!L.vox) {
    for (int k = 0; k < cnt; k++) {
      double t = daughter_dist_in(G, base + k, pl, vl, nc);
      saf = dmin(saf, daughter_safety_in(G, base + k, pl, nc));
      if (t < s) {
        s = t;
        lim = k;
      }
    }
    safety = saf;
    return s;
  }
  const double pc[3] = {pl.x, pl.y, pl.z};
  const double vc[3] = {vl.x, vl.y, vl.z};
  int idx[3];
#pragma unroll
  for (int a = 0; a < 3; a++) idx[a] = vox_axis_index(pc[a], L.vlo[a], L.vinv[a], L.n[a]);
  // safety also limited by the start node's faces (not beyond the grid edge)
#pragma unroll
  for (int a = 0; a < 3; a++) {
    double lo = L.vlo[a] + idx[a] * L.vw[a];
    double hi = L.vlo[a] + (idx[a] + 1) * L.vw[a];
    if (idx[a] > 0) saf = dmin(saf, dmax(pc[a] - lo, 0.0));
    if (idx[a] < L.n[a] - 1) saf = dmin(saf, dmax(hi - pc[a], 0.0));
  }
  bool first = true;
  for (;;) {
    int2 nd = G.vox_node[L.node_base + (idx[0] * L.n[1] + idx[1]) * L.n[2] + idx[2]];
    nc.node();
    if (first && start_node) *start_node = nd;
    if (ORDER != kOrderPlain && first && nd.y >= kOrderMinCand && L.wide) {
      const double rho = sqrt(pl.x * pl.x + pl.y * pl.y);
      int lead = -1;
      if (ORDER == kOrderLearned && pred >= 0 && pred < nd.y) lead = pred;
      if (lead < 0) {
        // the candidate nearest by its enclosing cylinder goes first
        double lbmin = kInf;
        for (int c = 0; c < nd.y; c++) {
          const double lb = cyl_bound(G.pv_cyl[base + G.vox_cand[nd.x + c]], rho, pl.z);
          if (lb < lbmin) {
            lbmin = lb;
            lead = c;
          }
        }
        if (lead < 0) lead = 0;
      }
      {
        int k = G.vox_cand[nd.x + lead];
        double t = daughter_dist_in(G, base + k, pl, vl, nc);
        saf = dmin(saf, daughter_safety_in(G, base + k, pl, nc));
        if (t < s || (t == s && lim >= 0 && k < lim)) {
          s = t;
          lim = k;
        }
      }
      for (int c = 0; c < nd.y; c++) {
        if (c == lead) continue;
        int k = G.vox_cand[nd.x + c];
        // skip, without fetching the candidate's records, when its enclosing
        // cylinder lies beyond the best distance (the cylinder distance also
        // serves as the candidate's share of the safety)
        const double lbc = cyl_bound(G.pv_cyl[base + k], rho, pl.z);
        if (lbc * (1.0 - 1e-12) > s + kTol) {
          saf = dmin(saf, lbc);
          continue;
        }
        const double sf = daughter_safety_in(G, base + k, pl, nc, true);
        saf = dmin(saf, sf);
        // skip when the candidate's safety or its bounding box lies beyond the best
        if (sf * (1.0 - 1e-12) > s + kTol || box_beyond(G.pv[base + k], pl, vl, s)) continue;
        double t = daughter_dist_in(G, base + k, pl, vl, nc, false);
        if (t < s || (t == s && lim >= 0 && k < lim)) {
          s = t;
          lim = k;
        }
      }
    } else {
      for (int c = 0; c < nd.y; c++) {
        int k = G.vox_cand[nd.x + c];
        double t = daughter_dist_in(G, base + k, pl, vl, nc);
        if (first) saf = dmin(saf, daughter_safety_in(G, base + k, pl, nc));
        if (t < s || (t == s && lim >= 0 && k < lim)) {
          s = t;
          lim = k;
        }
      }
    }
    first = false;
    // distance to the node's exit plane along each axis
    double tx = kInf;
    int ax = -1;
#pragma unroll
    for (int a = 0; a < 3; a++) {
      if (vc[a] == 0.0) continue;
      double plane = L.vlo[a] + (idx[a] + (vc[a] > 0 ? 1 : 0)) * L.vw[a];
      double ta = (plane - pc[a]) / vc[a];
      if (ta < tx) {
        tx = ta;
        ax = a;
      }
    }
    if (ax < 0 || s < tx) break;
    idx[ax] += vc[ax] > 0 ? 1 : -1;
    if (idx[ax] < 0 || idx[ax] >= L.n[ax]) break;
  }
  safety = saf;
  return s;
}

// ---------------------------------------------------------------------------
// FP32-distance navigation (Sec. 5 names FP64 throughput among the limits
// of the GPU port).  Positions, optical depths, point-in-volume decisions,
// the voxel walk and the tallies stay FP64; what moves to FP32 is the
// solid arithmetic of the daughter candidates, on coordinates local to each
// candidate.  Two forms:
//  * screened: FP32 entry distances rank a node's candidates; the first in
//    that order is evaluated in FP64, and every other candidate is
//    evaluated in FP64 unless a rigorous FP32 lower bound on its FP64
//    distance exceeds the best distance so far.  Skipped candidates can
//    neither beat nor tie the result, so limiter, step and every later
//    decision equal the FP64 path's.
//  * pure: the step is the FP32 distance itself (mother and daughters).
// ---------------------------------------------------------------------------

enum : int { kPrecFP64 = 0, kPrecScreened = 1, kPrecPure = 2 };

// Candidate frame in FP32: offset from the placement origin in FP64, then
// rounded and rotated in FP32.
__device__ __forceinline__ void xf_local_f(const PRecF& P, V3 pl, V3 vl, V3f& pd, V3f& vd) {
  float d0 = (float)(pl.x - P.t[0]), d1 = (float)(pl.y - P.t[1]), d2 = (float)(pl.z - P.t[2]);
  float v0 = (float)vl.x, v1 = (float)vl.y, v2 = (float)vl.z;
  if (P.kind == 0) {
    pd = V3f{d0, d1, d2};
    vd = V3f{v0, v1, v2};
    return;
  }
  const float* r = P.r;
  pd = V3f{r[0] * d0 + r[1] * d1 + r[2] * d2, r[3] * d0 + r[4] * d1 + r[5] * d2,
           r[6] * d0 + r[7] * d1 + r[8] * d2};
  vd = V3f{r[0] * v0 + r[1] * v1 + r[2] * v2, r[3] * v0 + r[4] * v1 + r[5] * v2,
           r[6] * v0 + r[7] * v1 + r[8] * v2};
}

// Isotropic safety of a candidate from its FP32 local point, lowered by a
// margin that covers the rounding of the local point (about 2^-24 per
// coordinate and 2^-22 after the rotation), of the parameters (2^-24) and
// of the solid function (a few 2^-24 of the magnitudes involved), with a
// factor 16 to spare: 2^-18 of (|p|_1 * (1 + |B|) + parameter scale).
__device__ __forceinline__ float safety_lo_f(const PRecF& P, V3f pd) {
  float d = solid_d<float>(P.info, P.par, pd);
  float m = 0x1p-18f * ((fabsf(pd.x) + fabsf(pd.y) + fabsf(pd.z)) * P.sgrow + P.sscale);
  d -= m;
  return d > 0.f ? d : 0.f;
}

// Rigorous lower bound on the FP64 entry distance of a candidate from the
// mother-frame ray (pl, vl): the larger of its lowered safety and the ray's
// entry into its bounding box grown by mu = 2^-20 (|p|_inf + box scale),
// which exceeds the rounding of the FP32 point and of each slab numerator
// sixteen-fold, so the computed entry is never later than the true one and
// a ray that meets the true box is never declared a miss.  +inf on a miss.
__device__ __forceinline__ double lower_bound_f(const PRecF& P, V3 pl, V3 vl, V3f pd) {
  const float pc[3] = {(float)pl.x, (float)pl.y, (float)pl.z};
  const float vc[3] = {(float)vl.x, (float)vl.y, (float)vl.z};
  float pm = fmaxf(fmaxf(fabsf(pc[0]), fabsf(pc[1])), fabsf(pc[2]));
  float mu = 0x1p-20f * (pm + P.bscale);
  float te = 0.f, tx = __builtin_inff();
#pragma unroll
  for (int a = 0; a < 3; a++) {
    float n1 = P.lo[a] - pc[a], n2 = P.hi[a] - pc[a];
    if (vc[a] == 0.f) {
      // parallel to the slab: a miss only if outside the grown slab (a ray
      // with a direction component below float range would enter it only
      // after a distance far beyond any mother's exit distance)
      if (n1 - mu > 0.f || n2 + mu < 0.f) return kInf;
      continue;
    }
    float t1, t2;
    if (vc[a] > 0.f) {
      t1 = (n1 - mu) / vc[a];
      t2 = (n2 + mu) / vc[a];
    } else {
      t1 = (n2 + mu) / vc[a];
      t2 = (n1 - mu) / vc[a];
    }
    te = fmaxf(te, t1);
    tx = fminf(tx, t2);
  }
  if (te > tx) return kInf;
  return dmax((double)te, (double)safety_lo_f(P, pd));
}

// ComputeStep with FP32 candidate arithmetic (see above).  `lv` indexes the
// FP32 parameter twins of the mother (pure form only).  The walk, the node
// faces of the safety and the tie rule are those of compute_step.
template <bool C, bool PURE>
__device__ __forceinline__ double compute_step_f32(const DevGeom& G, const LRec& L, int lv, V3 pl, V3 vl,
                                                   int& lim, double& safety, NavCount<C>& nc) {
  const int info = L.info;
  double s, saf;
  if (PURE) {
    const float* q = G.lv_parf + (size_t)lv * kSolidPar;
    V3f pf{(float)pl.x, (float)pl.y, (float)pl.z}, vf{(float)vl.x, (float)vl.y, (float)vl.z};
    s = (double)solid_dist_out<float>(info, q, pf, vf);
    float md = solid_d<float>(info, q, pf);
    saf = md < 0.f ? (double)(-md) : 0.0;
  } else {
    s = solid_dist_out(info, L.par, pl, vl);
    double md = solid_d(info, L.par, pl);
    saf = md < 0 ? -md : 0.0;
  }
  nc.out(info);
  nc.saf(info, false);
  lim = kLimMother;
  const int cnt = L.dau_cnt;
  if (cnt == 0) {
    safety = saf;
    return s;
  }
  const int base = L.dau_base;
  const bool vox = L.vox != 0;
  const double pc[3] = {pl.x, pl.y, pl.z};
  const double vc[3] = {vl.x, vl.y, vl.z};
  int idx[3] = {0, 0, 0};
  if (vox) {
#pragma unroll
    for (int a = 0; a < 3; a++) idx[a] = vox_axis_index(pc[a], L.vlo[a], L.vinv[a], L.n[a]);
#pragma unroll
    for (int a = 0; a < 3; a++) {
      double lo = L.vlo[a] + idx[a] * L.vw[a];
      double hi = L.vlo[a] + (idx[a] + 1) * L.vw[a];
      if (idx[a] > 0) saf = dmin(saf, dmax(pc[a] - lo, 0.0));
      if (idx[a] < L.n[a] - 1) saf = dmin(saf, dmax(hi - pc[a], 0.0));
    }
  }
  bool first = true;
  for (;;) {
    int2 nd = int2{0, cnt};
    if (vox) {
      nd = G.vox_node[L.node_base + (idx[0] * L.n[1] + idx[1]) * L.n[2] + idx[2]];
      nc.node();
    }
    auto slot = [&](int c) { return vox ? (int)G.vox_cand[nd.x + c] : c; };
    if (PURE) {
      for (int c = 0; c < nd.y; c++) {
        const int k = slot(c);
        const PRecF& P = G.pvf[base + k];
        V3f pd, vd;
        xf_local_f(P, pl, vl, pd, vd);
        double t = (double)solid_dist_in<float>(P.info, P.par, pd, vd);
        nc.in32(P.info);
        if (first) {
          nc.saf(P.info, false);
          float d = solid_d<float>(P.info, P.par, pd);
          saf = dmin(saf, d > 0.f ? (double)d : 0.0);
        }
        if (t < s || (t == s && lim >= 0 && k < lim)) {
          s = t;
          lim = k;
        }
      }
    } else if (nd.y < kScreenMinCand) {
      // too few candidates to gain from screening: FP64 as in compute_step
      for (int c = 0; c < nd.y; c++) {
        const int k = slot(c);
        double t = daughter_dist_in(G, base + k, pl, vl, nc);
        if (first) saf = dmin(saf, daughter_safety_in(G, base + k, pl, nc));
        if (t < s || (t == s && lim >= 0 && k < lim)) {
          s = t;
          lim = k;
        }
      }
    } else {
      // rank by the FP32 entry distance; the node's safety from lowered FP32 safeties
      int lead = -1;
      float tl = __builtin_inff();
      for (int c = 0; c < nd.y; c++) {
        const PRecF& P = G.pvf[base + slot(c)];
        V3f pd, vd;
        xf_local_f(P, pl, vl, pd, vd);
        float t = solid_dist_in<float>(P.info, P.par, pd, vd);
        nc.in32(P.info);
        if (first) {
          nc.saf(P.info, false);
          saf = dmin(saf, (double)safety_lo_f(P, pd));
        }
        if (t < tl) {
          tl = t;
          lead = c;
        }
      }
      if (lead >= 0) {
        const int k = slot(lead);
        double t = daughter_dist_in(G, base + k, pl, vl, nc);
        if (t < s || (t == s && lim >= 0 && k < lim)) {
          s = t;
          lim = k;
        }
      }
      for (int c = 0; c < nd.y; c++) {
        if (c == lead) continue;
        const int k = slot(c);
        const PRecF& P = G.pvf[base + k];
        V3f pd, vd;
        xf_local_f(P, pl, vl, pd, vd);
        double lb = lower_bound_f(P, pl, vl, pd);
        if (lb * (1.0 - 1e-6) - kTol > s) continue;
        double t = daughter_dist_in(G, base + k, pl, vl, nc);
        if (t < s || (t == s && lim >= 0 && k < lim)) {
          s = t;
          lim = k;
        }
      }
    }
    first = false;
    if (!vox) break;
    double tx = kInf;
    int ax = -1;
#pragma unroll
    for (int a = 0; a < 3; a++) {
      if (vc[a] == 0.0) continue;
      double plane = L.vlo[a] + (idx[a] + (vc[a] > 0 ? 1 : 0)) * L.vw[a];
      double ta = (plane - pc[a]) / vc[a];
      if (ta < tx) {
        tx = ta;
        ax = a;
      }
    }
    if (ax < 0 || s < tx) break;
    idx[ax] += vc[ax] > 0 ? 1 : -1;
    if (idx[ax] < 0 || idx[ax] >= L.n[ax]) break;
  }
  safety = saf;
  return s;
}

// Precision dispatch of ComputeStep.
template <bool C, int ORDER, int PREC>
__device__ __forceinline__ double compute_step_p(const DevGeom& G, const LRec& L, int lv, V3 pl, V3 vl,
                                                 int& lim, double& safety, NavCount<C>& nc, int pred,
                                                 int2* start_node) {
  if constexpr (PREC == kPrecFP64) {
    return compute_step<C, ORDER>(G, L, pl, vl, lim, safety, nc, pred, start_node);
  } else {
    if (start_node) *start_node = int2{0, 0};
    return compute_step_f32<C, PREC == kPrecPure>(G, L, lv, pl, vl, lim, safety, nc);
  }
}

// ---------------------------------------------------------------------------
// Random numbers: Philox4x32-10 keyed by (event, track key, draw)
// ---------------------------------------------------------------------------

struct Philox {
  uint32_t event, tkey;
  uint32_t draw;
  uint32_t blk = 0xFFFFFFFFu;  // block index held in w (draws 2k and 2k+1 share a block)
  uint32_t w[4] = {0, 0, 0, 0};
};

__device__ __forceinline__ void philox_block(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                             uint32_t k0, uint32_t k1, uint32_t out[4]) {
#pragma unroll
  for (int r = 0; r < 10; r++) {
    uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
    uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

__device__ __forceinline__ void rng_start(Philox& r, uint32_t event, uint32_t tkey) {
  r.event = event;
  r.tkey = tkey;
  r.draw = 0;
}

// Uniform in (0, 1]: draw n uses words 2(n&1), 2(n&1)+1 of Philox block n/2
// (counter {n/2, track key, event, 0}, key = seed); 53 bits plus one.
__device__ __forceinline__ double rng_next(Philox& r, uint32_t seed_lo, uint32_t seed_hi) {
  uint32_t b = r.draw >> 1;
  if (b != r.blk) {
    philox_block(b, r.tkey, r.event, 0u, seed_lo, seed_hi, r.w);
    r.blk = b;
  }
  uint32_t lo = (r.draw & 1u) ? r.w[2] : r.w[0];
  uint32_t hi = (r.draw & 1u) ? r.w[3] : r.w[1];
  r.draw++;
  uint64_t m = ((((uint64_t)hi) << 32) | (uint64_t)lo) >> 11;
  return (double)(m + 1u) * 0x1p-53;
}

}  // namespace gnav

// gnav_host.cpp -- host runtime behind the C ABI: geometry validation and
// flattening, touchable expansion, voxel grids, attenuation tables, device
// buffers, tallies and launches.
//
// Alg. 2 (Sec. 3.4) of the paper loads the geometry and copies it to the GPU
// once (phase 1) and times only the parallel phase; the same split holds here:
// everything in this file runs at upload time or around a launch, never per
// step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "gnav.h"
#include "gnav_device.h"
#include "gnav_internal.h"

using namespace gnav;

static constexpr int kSolidStride = 16;  // host-side staging of solid parameters

// Scratch of gnav_transport_batch_noalloc, one copy per device for the life of
// the process: the work-queue counter in the first kNoallocQueueBytes, then
// one pending-photon entry (6 doubles) per track-pool slot.  On the host this
// name is not a device address; host code uses only the address that
// hipGetSymbolAddress returns for the current device (scratch_address).
static constexpr size_t kNoallocQueueBytes = 256;
static constexpr size_t kNoallocBytes =
    kNoallocQueueBytes + (size_t)GNAV_NOALLOC_MAX_SLOTS * 6 * sizeof(double);
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

namespace {

// ---------------------------------------------------------------------------
// Device buffer
// ---------------------------------------------------------------------------

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  // Reallocate to n bytes (at least 8, so empty tables keep a valid
  // pointer) and fill from host memory src, or with zeros; the copy is
  // ordered on `stream` (the caller keeps src alive until the stream passes it).
  hipError_t upload(const void* src, size_t n, hipStream_t stream = nullptr) {
    release();
    if (n == 0) n = 8;
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) {
      p = nullptr;
      return e;
    }
    bytes = n;
    if (src) return hipMemcpyAsync(p, src, n, hipMemcpyHostToDevice, stream);
    return hipMemsetAsync(p, 0, n, stream);
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

template <class T>
hipError_t up(DevBuf& b, const std::vector<T>& v, hipStream_t stream) {
  return b.upload(v.empty() ? nullptr : v.data(), v.size() * sizeof(T), stream);
}

// ---------------------------------------------------------------------------
// Attenuation tables (per material, photoelectric / Compton / pair)
// ---------------------------------------------------------------------------

constexpr long double kRe = 2.8179403262e-13L;  // classical electron radius, cm
constexpr long double kNA = 6.02214076e23L;     // 1/mol
constexpr long double kAlpha = 1.0L / 137.035999084L;
constexpr long double kPi = 3.141592653589793238462643383279502884L;
constexpr long double kPeScale = 4.0e-32L;      // cm2 MeV^3 (4.0e-8 barn MeV^3)

// Klein-Nishina total cross section per electron (cm2), k = E / m_e c^2,
// evaluated in extended precision because its terms cancel at small k.
long double kn_total(long double k) {
  long double two_k = 2.0L * k;
  long double lg = log1pl(two_k);
  long double inv = 1.0L / (1.0L + two_k);
  long double t1 = (1.0L + k) / (k * k) * (2.0L * (1.0L + k) * inv - lg / k);
  long double t2 = lg / two_k;
  long double t3 = (1.0L + 3.0L * k) * inv * inv;
  return 2.0L * kPi * kRe * kRe * (t1 + t2 - t3);
}

// Per-atom cross sections (cm2): photoelectric K Z^4/E^3, Compton Z sigma_KN,
// and nuclear-field pair production alpha r_e^2 Z^2 F(k) with F the
// unscreened Bethe-Heitler form, raised to the near-threshold (k-2)^3 term and
// capped by complete screening.
void atom_xs(int Z, long double E, long double out[3]) {
  long double z = (long double)Z;
  long double k = E / (long double)kMe;
  out[0] = kPeScale * (z * z) * (z * z) / (E * E * E);
  out[1] = z * kn_total(k);
  out[2] = 0.0L;
  if (k > 2.0L) {
    long double r = 1.0L - 2.0L / k;
    long double thr = (2.0L * kPi / 3.0L) * r * r * r;
    long double bh = (28.0L / 9.0L) * logl(2.0L * k) - 218.0L / 27.0L;
    long double cs = (28.0L / 9.0L) * logl(183.0L / cbrtl(z)) - 2.0L / 27.0L;
    long double f = std::min(cs, std::max(thr, bh));
    out[2] = kAlpha * kRe * kRe * z * z * f;
  }
}

// ---------------------------------------------------------------------------
// Solid preprocessing and extents
// ---------------------------------------------------------------------------

struct Box3 {
  double lo[3], hi[3];
};

// Extent of a tube/cone section (local frame): the corners of the annular
// sector at its smallest and largest radius plus its axis crossings.
void sector_extent(double rmin1, double rmax1, double rmin2, double rmax2, double dz, double sphi,
                   double dphi, Box3* ext) {
  double rlo = std::min(rmin1, rmin2), rhi = std::max(rmax1, rmax2);
  ext->lo[2] = -dz;
  ext->hi[2] = dz;
  if (!(dphi < 2.0 * M_PI)) {
    ext->lo[0] = ext->lo[1] = -rhi;
    ext->hi[0] = ext->hi[1] = rhi;
    return;
  }
  double lx = INFINITY, hx = -INFINITY, ly = INFINITY, hy = -INFINITY;
  for (double r : {rlo, rhi}) {
    for (double a : {sphi, sphi + dphi}) {
      lx = std::min(lx, r * std::cos(a));
      hx = std::max(hx, r * std::cos(a));
      ly = std::min(ly, r * std::sin(a));
      hy = std::max(hy, r * std::sin(a));
    }
  }
  for (int k = -8; k <= 8; k++) {
    double a = k * 0.5 * M_PI;
    if (a > sphi && a < sphi + dphi) {
      lx = std::min(lx, rhi * std::cos(a));
      hx = std::max(hx, rhi * std::cos(a));
      ly = std::min(ly, rhi * std::sin(a));
      hy = std::max(hy, rhi * std::sin(a));
    }
  }
  ext->lo[0] = lx;
  ext->hi[0] = hx;
  ext->lo[1] = ly;
  ext->hi[1] = hy;
}

bool solid_prep(int type, const double* par, double* q /*16*/, int* info, Box3* ext, std::string& why) {
  for (int i = 0; i < kSolidStride; i++) q[i] = 0.0;
  for (int i = 0; i < 8; i++) {
    if (!std::isfinite(par[i])) {
      why = "non-finite solid parameter";
      return false;
    }
  }
  if (type == kBox) {
    if (!(par[0] > 0 && par[1] > 0 && par[2] > 0)) {
      why = "box half lengths must be positive";
      return false;
    }
    q[0] = par[0];
    q[1] = par[1];
    q[2] = par[2];
    *info = kBox;
    for (int a = 0; a < 3; a++) {
      ext->lo[a] = -par[a];
      ext->hi[a] = par[a];
    }
    return true;
  }
  if (type == kOrb) {
    if (!(par[0] > 0)) {
      why = "orb radius must be positive";
      return false;
    }
    q[0] = par[0];
    *info = kOrb;
    for (int a = 0; a < 3; a++) {
      ext->lo[a] = -par[0];
      ext->hi[a] = par[0];
    }
    return true;
  }
  if (type == kTrd) {
    // half widths dx1, dx2 (x at z = -dz, +dz), dy1, dy2, half length dz; the
    // x faces are the planes |x| = a + b z with a = (dx1 + dx2) / 2 and
    // b = (dx2 - dx1) / (2 dz), unit normal (+-1, 0, -b) / sqrt(1 + b^2)
    if (!(par[0] > 0 && par[1] > 0 && par[2] > 0 && par[3] > 0 && par[4] > 0)) {
      why = "trapezoid half lengths must be positive";
      return false;
    }
    const double dz = par[4];
    for (int ax = 0; ax < 2; ax++) {
      const double d1 = par[2 * ax], d2 = par[2 * ax + 1];
      const double a = 0.5 * (d1 + d2);
      const double b = (d2 - d1) / (2.0 * dz);
      const double c = 1.0 / std::sqrt(1.0 + b * b);
      q[3 * ax] = c;
      q[3 * ax + 1] = -b * c;
      q[3 * ax + 2] = a * c;
      ext->lo[ax] = -std::max(d1, d2);
      ext->hi[ax] = std::max(d1, d2);
    }
    q[6] = dz;
    ext->lo[2] = -dz;
    ext->hi[2] = dz;
    *info = kTrd;
    return true;
  }
  if (type == kSphere) {
    // rmin, rmax, sphi, dphi, stheta, dtheta: q = {rmax, rmin, phi plane normals,
    // B1, c1, B2, c2} (theta bound j as the cone rho = B z, B = tan theta,
    // c = 1 / sqrt(1 + B^2)), bound kinds in the info bits
    const double rmin = par[0], rmax = par[1], sp = par[2], dp = par[3], st = par[4], dt = par[5];
    const double twopi = 2.0 * M_PI;
    if (!(rmin >= 0) || !(rmax > rmin) || (rmin > 0 && rmin < kTol)) {
      why = "sphere radii out of range";
      return false;
    }
    if (!(dp > 0) || dp > twopi || (dp < twopi && dp > M_PI)) {
      why = "phi sections must span (0, pi] or the full 2 pi";
      return false;
    }
    if (!(st >= 0) || !(dt > 0) || st + dt > M_PI * (1.0 + 1e-15)) {
      why = "theta section must lie in [0, pi]";
      return false;
    }
    q[0] = rmax;
    q[1] = rmin;
    int inf = kSphere;
    if (rmin > 0) inf |= kInfoInner;
    if (dp < twopi) {
      inf |= kInfoPhi;
      const double ep = sp + dp;
      q[2] = std::sin(sp);
      q[3] = -std::cos(sp);
      q[4] = -std::sin(ep);
      q[5] = std::cos(ep);
    }
    const double th[2] = {st, st + dt};
    for (int j = 0; j < 2; j++) {
      const bool present = j == 0 ? th[0] > 0 : th[1] < M_PI;
      int kind = kTNone;
      if (present) {
        if (th[j] == 0.5 * M_PI) {
          kind = j == 0 ? kTZle : kTZge;
        } else {
          q[6 + 2 * j] = std::tan(th[j]);
          q[7 + 2 * j] = 1.0 / std::sqrt(1.0 + q[6 + 2 * j] * q[6 + 2 * j]);
          const bool lower_half = th[j] > 0.5 * M_PI;
          // theta >= th below the equator and theta <= th above it keep the
          // inside of the cone, the other two its outside
          kind = (j == 0) != lower_half ? kTInner : kTOuter;
        }
      }
      inf |= kind << (kInfoTheta + 3 * j);
    }
    *info = inf;
    for (int a = 0; a < 3; a++) {
      ext->lo[a] = -rmax;
      ext->hi[a] = rmax;
    }
    return true;
  }
  double rmin1, rmax1, rmin2, rmax2, dz, sphi, dphi;
  if (type == kTubs) {
    rmin1 = rmin2 = par[0];
    rmax1 = rmax2 = par[1];
    dz = par[2];
    sphi = par[3];
    dphi = par[4];
  } else if (type == kCons) {
    rmin1 = par[0];
    rmax1 = par[1];
    rmin2 = par[2];
    rmax2 = par[3];
    dz = par[4];
    sphi = par[5];
    dphi = par[6];
  } else {
    why = "unknown solid type";
    return false;
  }
  if (!(dz > 0) || !(rmin1 >= 0) || !(rmin2 >= 0) || !(rmax1 > rmin1) || !(rmax2 > rmin2)) {
    why = "section radii/half length out of range";
    return false;
  }
  if ((rmin1 > 0 && rmin1 < kTol) || (rmin2 > 0 && rmin2 < kTol)) {
    why = "inner radius below the surface tolerance";
    return false;
  }
  const double twopi = 2.0 * M_PI;
  if (!(dphi > 0) || dphi > twopi || (dphi < twopi && dphi > M_PI)) {
    why = "phi sections must span (0, pi] or the full 2 pi";
    return false;
  }
  q[R_AO] = 0.5 * (rmax1 + rmax2);
  q[R_BO] = (rmax2 - rmax1) / (2.0 * dz);
  q[R_CO] = 1.0 / std::sqrt(1.0 + q[R_BO] * q[R_BO]);
  q[R_AI] = 0.5 * (rmin1 + rmin2);
  q[R_BI] = (rmin2 - rmin1) / (2.0 * dz);
  q[R_CI] = 1.0 / std::sqrt(1.0 + q[R_BI] * q[R_BI]);
  q[R_DZ] = dz;
  int inf = type;
  if (rmin1 > 0 || rmin2 > 0) inf |= kInfoInner;
  bool phi = dphi < twopi;
  if (phi) {
    inf |= kInfoPhi;
    double ephi = sphi + dphi;
    q[R_NS0] = std::sin(sphi);
    q[R_NS1] = -std::cos(sphi);
    q[R_NE0] = -std::sin(ephi);
    q[R_NE1] = std::cos(ephi);
  }
  *info = inf;
  sector_extent(rmin1, rmax1, rmin2, rmax2, dz, sphi, dphi, ext);
  return true;
}

// Extent of a placed solid in its mother frame: the 8 transformed corners of
// the local extent (exact for axis-aligned placements, conservative otherwise).
Box3 place_box(const Box3& b, const double* R, const double* t) {
  Box3 o;
  for (int a = 0; a < 3; a++) {
    o.lo[a] = INFINITY;
    o.hi[a] = -INFINITY;
  }
  for (int c = 0; c < 8; c++) {
    double p[3] = {(c & 1) ? b.hi[0] : b.lo[0], (c & 2) ? b.hi[1] : b.lo[1], (c & 4) ? b.hi[2] : b.lo[2]};
    for (int a = 0; a < 3; a++) {
      double x = R[3 * a] * p[0] + R[3 * a + 1] * p[1] + R[3 * a + 2] * p[2] + t[a];
      o.lo[a] = std::min(o.lo[a], x);
      o.hi[a] = std::max(o.hi[a], x);
    }
  }
  return o;
}

// Tighter placed extent: a tube/cone section turned about z is the same
// section with its start angle shifted, so its extent is recomputed exactly.
Box3 place_solid(int type, const double* par, const Box3& local, const double* R, const double* t) {
  bool zrot = R[2] == 0.0 && R[5] == 0.0 && R[6] == 0.0 && R[7] == 0.0 && R[8] == 1.0;
  if (zrot && (type == kTubs || type == kCons)) {
    double th = std::atan2(R[3], R[0]);
    Box3 e;
    if (type == kTubs) sector_extent(par[0], par[1], par[0], par[1], par[2], par[3] + th, par[4], &e);
    else sector_extent(par[0], par[1], par[2], par[3], par[4], par[5] + th, par[6], &e);
    // guard against rounding of the shifted angle
    for (int a = 0; a < 3; a++) {
      double pad = 1e-9 * std::max(1.0, std::max(std::fabs(e.lo[a]), std::fabs(e.hi[a])));
      e.lo[a] += t[a] - pad;
      e.hi[a] += t[a] + pad;
    }
    Box3 loose = place_box(local, R, t);
    for (int a = 0; a < 3; a++) {
      e.lo[a] = std::max(e.lo[a], loose.lo[a]);
      e.hi[a] = std::min(e.hi[a], loose.hi[a]);
    }
    return e;
  }
  return place_box(local, R, t);
}

// True when the placement's extent is exact (axis-permuting rotation or a
// z-turned section), so a protrusion beyond the mother's extent is real.
bool extent_is_tight(int type, const double* R) {
  bool zrot = R[2] == 0.0 && R[5] == 0.0 && R[6] == 0.0 && R[7] == 0.0 && R[8] == 1.0;
  if (zrot && (type == kTubs || type == kCons)) return true;
  for (int i = 0; i < 9; i++)
    if (R[i] != 0.0 && R[i] != 1.0 && R[i] != -1.0) return false;
  return true;
}

// ---------------------------------------------------------------------------
// Voxel grids (the smart voxels of Sec. 3.2's navigation, uniform per
// mother).  Grid choice: per axis a slice count from a small candidate set;
// the score is the mean number of candidates per node plus a small
// per-slice walk cost.  The first search counts bounding-box overlaps
// (separable per daughter: sum of slice span products / nodes); mothers whose
// daughters' boxes overlap heavily (concentric shells) get a second search
// with shape-aware counts.  Node lists always hold exactly the daughters
// whose solid may meet the node (conservative shape test), not every
// daughter whose bounding box does.
// ---------------------------------------------------------------------------

struct VoxBuild {
  double lo[3], w[3], inv_w[3];
  int n[3];
  std::vector<std::vector<uint16_t>> nodes;
};

// A placed daughter as the voxel builder sees it: padded extent in the
// mother frame plus the solid itself, for shape-aware node lists.
struct DauShape {
  Box3 box;
  int info;
  double q[kSolidPar];
  double R[9];  // daughter -> mother rotation: x_mother = R x_local + t
  double t[3];
};

int span_lo(double x, double lo, double w, int n) {
  double f = std::floor((x - lo) / w);
  if (f < 0) return 0;
  if (f > n - 1) return n - 1;
  return (int)f;
}

// Conservative test: may the daughter's solid meet box b (mother frame)?
// The box goes to the daughter frame as the extent of its 8 transformed
// corners, grown by pad; boxes are tested slab-wise, orbs by the box's
// nearest point, tube and cone sections by the range of the distance to the
// axis over the box against the radii over the box's z range (phi sections
// are not used to reject).  A false "meets" only costs a candidate; a false
// "misses" never happens.
bool shape_meets_box(const DauShape& d, const Box3& b, double pad) {
  for (int a = 0; a < 3; a++)
    if (b.hi[a] < d.box.lo[a] || b.lo[a] > d.box.hi[a]) return false;
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int c = 0; c < 8; c++) {
    double p[3] = {((c & 1) ? b.hi[0] : b.lo[0]) - d.t[0], ((c & 2) ? b.hi[1] : b.lo[1]) - d.t[1],
                   ((c & 4) ? b.hi[2] : b.lo[2]) - d.t[2]};
    for (int i = 0; i < 3; i++) {
      double x = d.R[i] * p[0] + d.R[3 + i] * p[1] + d.R[6 + i] * p[2];  // R^T p
      lo[i] = std::min(lo[i], x);
      hi[i] = std::max(hi[i], x);
    }
  }
  for (int i = 0; i < 3; i++) {
    lo[i] -= pad;
    hi[i] += pad;
  }
  const double* q = d.q;
  switch (d.info & 15) {
    case kBox:
      for (int i = 0; i < 3; i++)
        if (hi[i] < -q[i] || lo[i] > q[i]) return false;
      return true;
    case kOrb: {
      double s2 = 0;
      for (int i = 0; i < 3; i++) {
        double e = lo[i] > 0 ? lo[i] : (hi[i] < 0 ? -hi[i] : 0.0);
        s2 += e * e;
      }
      return s2 <= q[0] * q[0];
    }
    case kSphere: {
      // the box against the shell: nearest point beyond rmax, or farthest
      // point inside rmin
      double n2 = 0, f2 = 0;
      for (int i = 0; i < 3; i++) {
        double e = lo[i] > 0 ? lo[i] : (hi[i] < 0 ? -hi[i] : 0.0);
        double f = std::max(std::fabs(lo[i]), std::fabs(hi[i]));
        n2 += e * e;
        f2 += f * f;
      }
      if (n2 > q[0] * q[0]) return false;
      if ((d.info & kInfoInner) && f2 < q[1] * q[1]) return false;
      return true;
    }
    case kTrd: {
      // separating face plane: every corner of the (padded, daughter-frame)
      // box outside one face plane n . p = h
      const double nrm[6][4] = {{q[0], 0.0, q[1], q[2]}, {-q[0], 0.0, q[1], q[2]}, {0.0, q[3], q[4], q[5]},
                                {0.0, -q[3], q[4], q[5]}, {0.0, 0.0, 1.0, q[6]}, {0.0, 0.0, -1.0, q[6]}};
      for (int f = 0; f < 6; f++) {
        double mn = 0.0;
        for (int a = 0; a < 3; a++) mn += nrm[f][a] * (nrm[f][a] > 0 ? lo[a] : hi[a]);
        if (mn > nrm[f][3]) return false;
      }
      return true;
    }
    default: {
      double dz = q[R_DZ];
      double z0 = std::max(lo[2], -dz), z1 = std::min(hi[2], dz);
      if (z0 > z1) return false;
      double ex = lo[0] > 0 ? lo[0] : (hi[0] < 0 ? -hi[0] : 0.0);
      double ey = lo[1] > 0 ? lo[1] : (hi[1] < 0 ? -hi[1] : 0.0);
      double rho_min = std::sqrt(ex * ex + ey * ey);
      double fx = std::max(std::fabs(lo[0]), std::fabs(hi[0]));
      double fy = std::max(std::fabs(lo[1]), std::fabs(hi[1]));
      double rho_max = std::sqrt(fx * fx + fy * fy);
      double r_out = q[R_AO] + q[R_BO] * (q[R_BO] > 0 ? z1 : z0);
      if (rho_min > r_out) return false;
      if (d.info & kInfoInner) {
        double r_in = q[R_AI] + q[R_BI] * (q[R_BI] > 0 ? z0 : z1);
        if (rho_max < r_in) return false;
      }
      return true;
    }
  }
}

// Node box of grid (lo, w) at index (i, j, k), grown by pad.
Box3 node_box(const double* lo, const double* w, int i, int j, int k, double pad) {
  Box3 b;
  const int ix[3] = {i, j, k};
  for (int a = 0; a < 3; a++) {
    b.lo[a] = lo[a] + ix[a] * w[a] - pad;
    b.hi[a] = lo[a] + (ix[a] + 1) * w[a] + pad;
  }
  return b;
}

// Mean candidates per node of grid n over box g with shape-aware lists:
// every node when there are at most 512, else a fixed pseudo-random sample.
double shape_cost(const Box3& g, const int* n, const std::vector<DauShape>& dau, double pad) {
  double w[3];
  for (int a = 0; a < 3; a++) w[a] = (g.hi[a] - g.lo[a]) / n[a];
  const long total = (long)n[0] * n[1] * n[2];
  const long samples = std::min<long>(total, 512);
  uint64_t h = 0x9E3779B97F4A7C15ull;
  double sum = 0;
  for (long s = 0; s < samples; s++) {
    long id = s;
    if (samples < total) {
      h ^= h << 13;
      h ^= h >> 7;
      h ^= h << 17;
      id = (long)(h % (uint64_t)total);
    }
    int i = (int)(id / ((long)n[1] * n[2])), j = (int)((id / n[2]) % n[1]), k = (int)(id % n[2]);
    Box3 b = node_box(g.lo, w, i, j, k, pad);
    for (const DauShape& d : dau) sum += shape_meets_box(d, b, pad) ? 1.0 : 0.0;
  }
  return sum / samples;
}

VoxBuild build_voxels(const Box3& mother, const std::vector<DauShape>& dau, bool shape_aware) {
  const int cnt = (int)dau.size();
  Box3 g = mother;
  for (const DauShape& d : dau) {
    for (int a = 0; a < 3; a++) {
      g.lo[a] = std::min(g.lo[a], d.box.lo[a]);
      g.hi[a] = std::max(g.hi[a], d.box.hi[a]);
    }
  }
  // pad the grid box slightly so points on its faces map inside
  double scale = 1.0;
  for (int a = 0; a < 3; a++) {
    double s = 1e-9 * std::max(1.0, std::max(std::fabs(g.lo[a]), std::fabs(g.hi[a])));
    g.lo[a] -= s;
    g.hi[a] += s;
    scale = std::max(scale, std::max(std::fabs(g.lo[a]), std::fabs(g.hi[a])));
  }
  // node boxes are grown by pad before the shape test (well above the
  // surface tolerance, so surface points find their daughters)
  const double pad = 1e-6 + 1e-12 * scale;
  const int max_nodes = std::max(64, std::min(1 << 18, 8 * cnt));
  std::vector<int> opts[3];
  for (int a = 0; a < 3; a++) {
    std::vector<double> w;
    for (const DauShape& d : dau) w.push_back(d.box.hi[a] - d.box.lo[a]);
    std::nth_element(w.begin(), w.begin() + w.size() / 2, w.end());
    double med = std::max(w[w.size() / 2], 1e-6);
    double L = g.hi[a] - g.lo[a];
    std::vector<int> o = {1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128};
    for (double f : {1.0, 2.0}) {
      long m = std::lround(f * L / med);
      if (m >= 1 && m <= 256) o.push_back((int)m);
    }
    std::sort(o.begin(), o.end());
    o.erase(std::unique(o.begin(), o.end()), o.end());
    opts[a] = o;
  }
  // bounding-box cost: spans[a][option][daughter]
  std::vector<std::vector<std::vector<int>>> spans(3);
  for (int a = 0; a < 3; a++) {
    for (int n : opts[a]) {
      double w = (g.hi[a] - g.lo[a]) / n;
      std::vector<int> s(cnt);
      for (int d = 0; d < cnt; d++) {
        s[d] = span_lo(dau[d].box.hi[a], g.lo[a], w, n) - span_lo(dau[d].box.lo[a], g.lo[a], w, n) + 1;
      }
      spans[a].push_back(std::move(s));
    }
  }
  double best = INFINITY, best_cand = 0;
  int bn[3] = {1, 1, 1};
  for (size_t i = 0; i < opts[0].size(); i++)
    for (size_t j = 0; j < opts[1].size(); j++)
      for (size_t k = 0; k < opts[2].size(); k++) {
        long nodes = (long)opts[0][i] * opts[1][j] * opts[2][k];
        if (nodes > max_nodes) continue;
        double tot = 0;
        for (int d = 0; d < cnt; d++)
          tot += (double)spans[0][i][d] * spans[1][j][d] * spans[2][k][d];
        double score = tot / nodes + 0.02 * (opts[0][i] + opts[1][j] + opts[2][k]);
        if (score < best - 1e-12) {
          best = score;
          best_cand = tot / nodes;
          bn[0] = opts[0][i];
          bn[1] = opts[1][j];
          bn[2] = opts[2][k];
        }
      }
  // Daughters whose bounding boxes overlap heavily (nested shells, sections
  // around an axis) leave many candidates per node: then search again with
  // shape-aware counts over power-of-two grids, allowing finer grids.
  if (shape_aware && best_cand > 4.0) {
    double cur = shape_cost(g, bn, dau, pad) + 0.02 * (bn[0] + bn[1] + bn[2]);
    const long max_fine = std::max<long>(max_nodes, std::min<long>(1 << 16, 64L * cnt));
    const int ladder[] = {1, 2, 4, 8, 16, 32, 64, 128};
    for (int nx : ladder)
      for (int ny : ladder)
        for (int nz : ladder) {
          if ((long)nx * ny * nz > max_fine) continue;
          const int n3[3] = {nx, ny, nz};
          double score = 0.02 * (nx + ny + nz);
          if (score >= cur) continue;
          score += shape_cost(g, n3, dau, pad);
          if (score < cur - 1e-12) {
            cur = score;
            bn[0] = nx;
            bn[1] = ny;
            bn[2] = nz;
          }
        }
  }
  VoxBuild vb;
  for (int a = 0; a < 3; a++) {
    vb.n[a] = bn[a];
    vb.lo[a] = g.lo[a];
    vb.w[a] = (g.hi[a] - g.lo[a]) / bn[a];
    vb.inv_w[a] = 1.0 / vb.w[a];
  }
  const int nx = vb.n[0], ny = vb.n[1], nz = vb.n[2];
  vb.nodes.assign((size_t)nx * ny * nz, {});
  for (int d = 0; d < cnt; d++) {
    int l[3], h[3];
    for (int a = 0; a < 3; a++) {
      l[a] = span_lo(dau[d].box.lo[a], g.lo[a], vb.w[a], vb.n[a]);
      h[a] = span_lo(dau[d].box.hi[a], g.lo[a], vb.w[a], vb.n[a]);
    }
    for (int i = l[0]; i <= h[0]; i++)
      for (int j = l[1]; j <= h[1]; j++)
        for (int k = l[2]; k <= h[2]; k++)
          if (!shape_aware || shape_meets_box(dau[d], node_box(vb.lo, vb.w, i, j, k, pad), pad))
            vb.nodes[((size_t)i * ny + j) * nz + k].push_back((uint16_t)d);
  }
  return vb;
}

// ---------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------

struct GeomRec {
  gnav_mlp* mlp = nullptr;  // network for the learned candidate order
  uint64_t mlp_gen = 0;     // bumped whenever the binding changes
  int t_base, n_t;
  int n_class = 0;  // voxelised mothers (candidate-ordering classes)
  bool axis_boxes = false;  // every solid is a box and every placement a translation
  bool spheres = false;     // some solid is a sphere section
  bool any_wide = false;    // some mother's voxel nodes hold enough candidates for ordered walks
  int lv_base, pv_base, solid_base, mat_base;
  std::vector<int> h_parent, h_pv, h_lv, h_depth;  // per-geometry ids
};

}  // namespace

struct gnav_ctx {
  int device = 0;
  int n_cu = 256;
  std::string err;
  // concatenated host tables (records)
  std::vector<TRec> t_rec;
  std::vector<double> t_xf;
  std::vector<LRec> lv_rec;
  std::vector<PRec> pv_rec;
  std::vector<PRecF> pvf;
  std::vector<float4> pv_cyl;
  std::vector<float> lv_parf;
  std::vector<int2> vox_node;
  std::vector<uint16_t> vox_cand;
  std::vector<double> xs;
  std::vector<double> mat_rho;
  std::vector<GeomRec> geoms;
  std::vector<int> geom_tbase;
  int n_mats_total = 0;
  double lnE0 = 0, dlnE = 0;
  // device copies
  DevBuf d_t_rec, d_t_xf, d_lv_rec, d_pv_rec, d_pvf, d_pv_cyl, d_lv_parf, d_vox_node, d_vox_cand, d_xs,
      d_mat_rho, d_geom_tbase, d_nbr;
  DevBuf d_queue, d_pend, d_claim;
  DevGeom G{};
  // Generations of what a captured graph holds: the resident tables (every
  // upload reallocates them) and the launch buffers (the pending-photon
  // buffer, reallocated when a batch needs a larger grid, and the claim
  // order, reallocated when a batch holds more primaries).
  uint64_t tables_gen = 0, pend_gen = 0;
  // Launches of one context share d_queue and d_pend: a launch on another
  // stream than the previous one waits for it on the device.
  hipEvent_t last_launch = nullptr;
  hipStream_t last_stream = nullptr;
  bool launched = false;
  // autotuned launch settings by (geometry, precision, order, log2 of the batch size)
  std::map<std::array<int, 4>, gnav_tuning> tuning;
  // this device's copy of the no-allocation scratch array
  void* scratch = nullptr;
};

struct gnav_tally {
  int n_events = 0;
  int n_touch = 0;
  DevBuf edep_t, edep_ev, esc_ev, counters;
};

namespace {

// The four tally arrays zeroed in one launch (a kernel, so a graph can hold it).
hipError_t zero_tally(gnav_tally* t, hipStream_t st) {
  void* const p[4] = {t->edep_t.p, t->edep_ev.p, t->esc_ev.p, t->counters.p};
  const size_t w[4] = {t->edep_t.bytes / 8, t->edep_ev.bytes / 8, t->esc_ev.bytes / 8, t->counters.bytes / 8};
  return launch_zero4(p, w, st);
}

gnav_status fail(gnav_ctx* c, gnav_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

gnav_status hip_fail(gnav_ctx* c, hipError_t e, const char* what) {
  return fail(c, e == hipErrorOutOfMemory ? GNAV_ENOMEM : GNAV_EHIP,
              std::string(what) + ": " + hipGetErrorString(e));
}

// Device address of `scratch` on `device` (which must be current), looked up
// once per device and kept for the process.
hipError_t scratch_address(int device, void** out) {
  static std::mutex mu;
  static std::map<int, void*> addr;
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(device);
  if (it == addr.end()) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    it = addr.emplace(device, p).first;
  }
  *out = it->second;
  return hipSuccess;
}

#define HIP_TRY(ctx, expr, what)                     \
  do {                                               \
    hipError_t _e = (expr);                          \
    if (_e != hipSuccess) return hip_fail(ctx, _e, what); \
  } while (0)

// Face neighbours of box touchables (G.nbr), the relocation shortcut: for
// each face of each box touchable other than a world, the touchable that
// LocateGlobalPoint finds 1e-6 mm outside the face's centre, moving outward
// (global id), or -1 when that is outside the world or an ancestor of the
// box.  An ancestor is no shortcut: the relocation searches it with the box
// excluded, and the box may still pass its own inside test at a point its
// exit distance put on the face (within the tolerance), so a search that
// did not exclude it could return to it.  A hint only: the transport uses it
// after checking that the neighbour holds the crossing point.
hipError_t build_face_neighbours(gnav_ctx* c, hipStream_t stream) {
  const int nt = (int)c->t_rec.size();
  std::vector<int> nbr((size_t)nt * 6, -1);
  std::vector<double> pos, dir;
  std::vector<int> slot;  // index into nbr of each query
  constexpr double kOutside = 1e-6;
  hipError_t e = hipSuccess;
  for (const GeomRec& g : c->geoms) {
    pos.clear();
    dir.clear();
    slot.clear();
    for (int i = 1; i < g.n_t; i++) {
      const int T = g.t_base + i;
      const LRec& L = c->lv_rec[c->t_rec[T].lv];
      if ((L.info & 15) != kBox) continue;
      const double* m = &c->t_xf[(size_t)T * 12];  // local = M (x - t)
      for (int f = 0; f < 6; f++) {
        const int a = f / 2;
        const double sg = (f & 1) ? 1.0 : -1.0;
        double ql[3] = {0.0, 0.0, 0.0}, vl[3] = {0.0, 0.0, 0.0};
        ql[a] = sg * (L.par[a] + kOutside);
        vl[a] = sg;
        for (int r = 0; r < 3; r++) {  // x = M^T local + t (M orthonormal)
          pos.push_back(m[r] * ql[0] + m[3 + r] * ql[1] + m[6 + r] * ql[2] + m[9 + r]);
          dir.push_back(m[r] * vl[0] + m[3 + r] * vl[1] + m[6 + r] * vl[2]);
        }
        slot.push_back(T * 6 + f);
      }
    }
    const long n = (long)slot.size();
    if (n == 0) continue;
    DevBuf dp, dd, dout;
    if ((e = dp.upload(pos.data(), pos.size() * sizeof(double), stream)) != hipSuccess) return e;
    if ((e = dd.upload(dir.data(), dir.size() * sizeof(double), stream)) != hipSuccess) return e;
    if ((e = dout.upload(nullptr, n * sizeof(int), stream)) != hipSuccess) return e;
    if ((e = launch_locate(c->G, g.t_base, g.t_base, n, dp.as<double>(), dd.as<double>(), dout.as<int>(), stream)) !=
        hipSuccess)
      return e;
    std::vector<int> out(n);
    if ((e = hipMemcpyAsync(out.data(), dout.p, n * sizeof(int), hipMemcpyDeviceToHost, stream)) != hipSuccess)
      return e;
    if ((e = hipStreamSynchronize(stream)) != hipSuccess) return e;
    for (long q = 0; q < n; q++) {
      if (out[q] < 0) continue;
      const int N = g.t_base + out[q];
      int A = c->t_rec[slot[q] / 6].parent;
      while (A >= 0 && A != N) A = c->t_rec[A].parent;
      if (A < 0) nbr[slot[q]] = N;
    }
  }
  if ((e = up(c->d_nbr, nbr, stream)) != hipSuccess) return e;
  c->G.nbr = c->d_nbr.as<int>();
  return hipStreamSynchronize(stream);
}

hipError_t upload_all(gnav_ctx* c, hipStream_t stream) {
  hipError_t e;
  c->tables_gen++;
#define UP(buf, vec) \
  if ((e = up(c->buf, c->vec, stream)) != hipSuccess) return e;
  UP(d_t_rec, t_rec)
  UP(d_t_xf, t_xf)
  UP(d_lv_rec, lv_rec)
  UP(d_pv_rec, pv_rec)
  UP(d_pvf, pvf)
  UP(d_pv_cyl, pv_cyl)
  UP(d_lv_parf, lv_parf)
  UP(d_vox_node, vox_node)
  UP(d_vox_cand, vox_cand)
  UP(d_xs, xs)
  UP(d_mat_rho, mat_rho)
  UP(d_geom_tbase, geom_tbase)
#undef UP
  DevGeom& G = c->G;
  G.t = c->d_t_rec.as<TRec>();
  G.t_xf = c->d_t_xf.as<double>();
  G.lv = c->d_lv_rec.as<LRec>();
  G.pv = c->d_pv_rec.as<PRec>();
  G.pvf = c->d_pvf.as<PRecF>();
  G.pv_cyl = c->d_pv_cyl.as<float4>();
  G.lv_parf = c->d_lv_parf.as<float>();
  G.vox_node = c->d_vox_node.as<int2>();
  G.vox_cand = c->d_vox_cand.as<uint16_t>();
  G.xs = c->d_xs.as<double>();
  G.mat_rho = c->d_mat_rho.as<double>();
  G.lnE0 = c->lnE0;
  G.dlnE = c->dlnE;
  G.nbr = nullptr;
  if ((e = hipStreamSynchronize(stream)) != hipSuccess) return e;
  return build_face_neighbours(c, stream);
}

// Nearest float not above / not below x.
float round_down_f(double x) {
  float f = (float)x;
  if ((double)f > x) f = std::nextafter(f, -std::numeric_limits<float>::infinity());
  return f;
}

float round_up_f(double x) {
  float f = (float)x;
  if ((double)f < x) f = std::nextafter(f, std::numeric_limits<float>::infinity());
  return f;
}

// Enclosing annular cylinder {rho min, rho max, z min, z max} of a placed
// solid about its mother's z axis, rounded outward: from the padded placed
// bounding box, tightened by the solid's own radii for tube and cone sections
// on the mother's axis (rotations about z, or a flip of z) and for orbs.
float4 placed_cylinder(int type, const double* par, const double* R, const double* t, const PRec& pr) {
  const double* lo = pr.box_lo;
  const double* hi = pr.box_hi;
  double ex = lo[0] > 0 ? lo[0] : (hi[0] < 0 ? -hi[0] : 0.0);
  double ey = lo[1] > 0 ? lo[1] : (hi[1] < 0 ? -hi[1] : 0.0);
  double fx = std::max(std::fabs(lo[0]), std::fabs(hi[0]));
  double fy = std::max(std::fabs(lo[1]), std::fabs(hi[1]));
  double rmin = std::sqrt(ex * ex + ey * ey), rmax = std::sqrt(fx * fx + fy * fy);
  const double pad = 1e-7 + 1e-12 * std::max(rmax, std::max(std::fabs(lo[2]), std::fabs(hi[2])));
  const bool zaxis = R[2] == 0.0 && R[5] == 0.0 && R[6] == 0.0 && R[7] == 0.0 && std::fabs(R[8]) == 1.0;
  if ((type == kTubs || type == kCons) && zaxis && t[0] == 0.0 && t[1] == 0.0) {
    double r_in = type == kTubs ? par[0] : std::min(par[0], par[2]);
    double r_out = type == kTubs ? par[1] : std::max(par[1], par[3]);
    rmin = std::max(rmin, r_in - pad);
    rmax = std::min(rmax, r_out + pad);
  } else if (type == kOrb) {
    double rt = std::sqrt(t[0] * t[0] + t[1] * t[1]);
    rmin = std::max(rmin, rt - par[0] - pad);
    rmax = std::min(rmax, rt + par[0] + pad);
  }
  float4 c;
  c.x = round_down_f(std::max(rmin, 0.0));
  c.y = round_up_f(rmax);
  c.z = round_down_f(lo[2]);
  c.w = round_up_f(hi[2]);
  return c;
}

bool is_identity(const double* R) {
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++)
      if (R[3 * i + j] != (i == j ? 1.0 : 0.0)) return false;
  return true;
}

gnav_status check_geom(gnav_ctx* c, int geom_id) {
  if (!c) return GNAV_EINVAL;
  if (c->geoms.empty()) return fail(c, GNAV_ESTATE, "no geometry uploaded");
  if (geom_id < 0 || geom_id >= (int)c->geoms.size()) return fail(c, GNAV_EINVAL, "bad geometry id");
  return GNAV_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" {

gnav_status gnav_create(int32_t device, gnav_ctx** out) {
  if (!out) return GNAV_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return GNAV_EHIP;
  if (device < 0 || device >= ndev) return GNAV_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return GNAV_EHIP;
  gnav_ctx* c = new (std::nothrow) gnav_ctx();
  if (!c) return GNAV_ENOMEM;
  c->device = device;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
    c->n_cu = prop.multiProcessorCount;
  // the pending-photon buffer sized for the largest default grid (every pool
  // size fills the same slot count), so default batches never reallocate it
  const size_t pend_bytes = (size_t)c->n_cu * 3 * 256 * 6 * sizeof(double);
  if (c->d_queue.upload(nullptr, 64) != hipSuccess || c->d_pend.upload(nullptr, pend_bytes) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess) {
    delete c;
    return GNAV_ENOMEM;
  }
  if (hipEventCreateWithFlags(&c->last_launch, hipEventDisableTiming) != hipSuccess) {
    delete c;
    return GNAV_EHIP;
  }
  if (scratch_address(device, &c->scratch) != hipSuccess) {
    (void)hipEventDestroy(c->last_launch);
    delete c;
    return GNAV_EHIP;
  }
  c->lnE0 = std::log(1e-3);
  c->dlnE = std::log(1e5) / 256.0;
  *out = c;
  return GNAV_OK;
}

void gnav_destroy(gnav_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  if (ctx->last_launch) (void)hipEventDestroy(ctx->last_launch);
  delete ctx;
}

const char* gnav_last_error(const gnav_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

gnav_status gnav_upload_geometry(gnav_ctx* c, const gnav_geometry_desc* d, int32_t* geom_id,
                                 int32_t* n_touchables, void* stream) {
  if (!c || !d) return GNAV_EINVAL;
  c->err.clear();
  if (d->n_solids <= 0 || d->n_lv <= 0 || d->n_mats <= 0 || d->n_pv < 0)
    return fail(c, GNAV_EGEOM, "empty geometry");
  if (!d->solid_type || !d->solid_par || !d->mat_density || !d->mat_el_off || !d->lv_solid ||
      !d->lv_mat || !d->lv_dau_off || !d->lv_dau_cnt || (d->n_pv > 0 && (!d->pv_lv || !d->pv_rot ||
                                                                          !d->pv_trans)))
    return fail(c, GNAV_EINVAL, "null array in geometry description");
  if (d->world_lv < 0 || d->world_lv >= d->n_lv) return fail(c, GNAV_EGEOM, "bad world LV");
  if (d->voxel_lists != 0 && d->voxel_lists != 1) return fail(c, GNAV_EINVAL, "voxel_lists must be 0 or 1");
  // solids
  std::vector<double> q(d->n_solids * kSolidStride);
  std::vector<int> info(d->n_solids);
  std::vector<Box3> ext(d->n_solids);
  for (int s = 0; s < d->n_solids; s++) {
    std::string why;
    if (!solid_prep(d->solid_type[s], d->solid_par + 8 * s, &q[s * kSolidStride], &info[s], &ext[s], why))
      return fail(c, GNAV_EGEOM, "solid " + std::to_string(s) + ": " + why);
  }
  // materials
  int n_el = d->mat_el_off[d->n_mats];
  if (d->mat_el_off[0] != 0 || n_el < 0) return fail(c, GNAV_EGEOM, "bad material element ranges");
  if (n_el > 0 && (!d->el_Z || !d->el_A || !d->el_wfrac)) return fail(c, GNAV_EINVAL, "null element arrays");
  for (int m = 0; m < d->n_mats; m++) {
    if (!(d->mat_density[m] >= 0) || !std::isfinite(d->mat_density[m]))
      return fail(c, GNAV_EGEOM, "bad density");
    if (d->mat_el_off[m + 1] < d->mat_el_off[m]) return fail(c, GNAV_EGEOM, "bad material element ranges");
  }
  for (int e = 0; e < n_el; e++) {
    if (d->el_Z[e] < 1 || d->el_Z[e] > 120 || !(d->el_A[e] > 0) || !(d->el_wfrac[e] >= 0))
      return fail(c, GNAV_EGEOM, "bad element");
  }
  // LVs and PVs
  for (int l = 0; l < d->n_lv; l++) {
    if (d->lv_solid[l] < 0 || d->lv_solid[l] >= d->n_solids || d->lv_mat[l] < 0 || d->lv_mat[l] >= d->n_mats)
      return fail(c, GNAV_EGEOM, "LV " + std::to_string(l) + ": bad solid or material index");
    if (d->lv_dau_cnt[l] < 0 || d->lv_dau_off[l] < 0 || d->lv_dau_off[l] + d->lv_dau_cnt[l] > d->n_pv)
      return fail(c, GNAV_EGEOM, "LV " + std::to_string(l) + ": daughter range out of bounds");
    if (d->lv_dau_cnt[l] > 65535) return fail(c, GNAV_EGEOM, "more than 65535 daughters in one LV");
  }
  for (int p = 0; p < d->n_pv; p++) {
    if (d->pv_lv[p] < 0 || d->pv_lv[p] >= d->n_lv) return fail(c, GNAV_EGEOM, "PV: bad LV index");
    const double* R = d->pv_rot + 9 * p;
    for (int i = 0; i < 3; i++) {
      if (!std::isfinite(d->pv_trans[3 * p + i])) return fail(c, GNAV_EGEOM, "PV: non-finite translation");
      for (int j = 0; j < 3; j++) {
        double dot = 0;
        for (int k = 0; k < 3; k++) dot += R[3 * k + i] * R[3 * k + j];
        if (!(std::fabs(dot - (i == j ? 1.0 : 0.0)) < 1e-9))
          return fail(c, GNAV_EGEOM, "PV " + std::to_string(p) + ": rotation is not orthonormal");
      }
    }
  }
  // daughters must lie inside their mother's extent (conservative check)
  for (int l = 0; l < d->n_lv; l++) {
    const Box3& M = ext[d->lv_solid[l]];
    for (int k = 0; k < d->lv_dau_cnt[l]; k++) {
      int p = d->lv_dau_off[l] + k;
      int ds = d->lv_solid[d->pv_lv[p]];
      if (!extent_is_tight(d->solid_type[ds], d->pv_rot + 9 * p)) continue;
      Box3 b = place_solid(d->solid_type[ds], d->solid_par + 8 * ds, ext[ds], d->pv_rot + 9 * p,
                           d->pv_trans + 3 * p);
      for (int a = 0; a < 3; a++) {
        double slack = 1e-6 * std::max(1.0, std::fabs(M.hi[a] - M.lo[a]));
        if (b.lo[a] < M.lo[a] - slack || b.hi[a] > M.hi[a] + slack)
          return fail(c, GNAV_EGEOM, "LV " + std::to_string(l) + ": daughter " + std::to_string(k) +
                                         " protrudes from its mother");
      }
    }
  }
  // touchable count (fails on cycles / explosion)
  std::vector<long long> cnt(d->n_lv, 0);
  for (int it = 0; it <= d->n_lv + 1; it++) {
    bool changed = false;
    for (int l = 0; l < d->n_lv; l++) {
      long long s = 1;
      for (int k = 0; k < d->lv_dau_cnt[l]; k++) s += cnt[d->pv_lv[d->lv_dau_off[l] + k]];
      s = std::min(s, 1LL << 40);
      if (s != cnt[l]) {
        cnt[l] = s;
        changed = true;
      }
    }
    if (!changed) break;
    if (it == d->n_lv + 1) return fail(c, GNAV_EGEOM, "placement cycle");
  }
  long long nt_ll = cnt[d->world_lv];
  long long total_t = (long long)c->t_rec.size() + nt_ll;
  if (nt_ll > (1LL << 30) || total_t > (1LL << 30)) return fail(c, GNAV_EGEOM, "too many touchables");
  const int nt = (int)nt_ll;

  GeomRec gr;
  gr.t_base = (int)c->t_rec.size();
  gr.axis_boxes = std::all_of(d->solid_type, d->solid_type + d->n_solids, [](int32_t ty) { return ty == kBox; });
  gr.spheres = std::any_of(d->solid_type, d->solid_type + d->n_solids, [](int32_t ty) { return ty == kSphere; });
  for (int p = 0; p < d->n_pv && gr.axis_boxes; p++) gr.axis_boxes = is_identity(d->pv_rot + 9L * p);
  gr.n_t = nt;
  gr.lv_base = (int)c->lv_rec.size();
  gr.pv_base = (int)c->pv_rec.size();
  gr.solid_base = 0;
  gr.mat_base = c->n_mats_total;

  // attenuation tables per material
  for (int m = 0; m < d->n_mats; m++) {
    for (int p = 0; p < 3; p++) {
      for (int i = 0; i < kNNode; i++) {
        long double E = expl((long double)c->lnE0 + (long double)i * (long double)c->dlnE);
        long double mu = 0.0L;
        for (int e = d->mat_el_off[m]; e < d->mat_el_off[m + 1]; e++) {
          long double xsv[3];
          atom_xs(d->el_Z[e], (long double)(double)E, xsv);
          long double n_at = (long double)d->mat_density[m] * kNA * (long double)d->el_wfrac[e] /
                             (long double)d->el_A[e];
          mu += n_at * xsv[p];
        }
        c->xs.push_back((double)(mu * 0.1L));  // 1/cm -> 1/mm
      }
    }
  }
  for (int m = 0; m < d->n_mats; m++) c->mat_rho.push_back(d->mat_density[m]);
  c->n_mats_total += d->n_mats;
  // placements: M = R^T (row major, M[i][j] = R[j][i]) and t
  for (int p = 0; p < d->n_pv; p++) {
    const double* R = d->pv_rot + 9 * p;
    const double* t = d->pv_trans + 3 * p;
    PRec pr;
    std::memset(&pr, 0, sizeof(pr));
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++) pr.m[3 * i + j] = R[3 * j + i];
    pr.m[9] = t[0];
    pr.m[10] = t[1];
    pr.m[11] = t[2];
    pr.kind = is_identity(R) ? 0 : 1;
    pr.lv = gr.lv_base + d->pv_lv[p];
    {
      int ds = d->lv_solid[d->pv_lv[p]];
      Box3 b = place_solid(d->solid_type[ds], d->solid_par + 8 * ds, ext[ds], R, t);
      for (int a = 0; a < 3; a++) {
        double pad = 1e-7 + 1e-12 * std::max(std::fabs(b.lo[a]), std::fabs(b.hi[a]));
        pr.box_lo[a] = b.lo[a] - pad;
        pr.box_hi[a] = b.hi[a] + pad;
      }
    }
    c->pv_rec.push_back(pr);
    c->pv_cyl.push_back(placed_cylinder(d->solid_type[d->lv_solid[d->pv_lv[p]]],
                                        d->solid_par + 8 * d->lv_solid[d->pv_lv[p]], R, t, pr));
  }
  // logical volumes with their solid and voxel grid
  for (int l = 0; l < d->n_lv; l++) {
    LRec lr;
    std::memset(&lr, 0, sizeof(lr));
    int s = d->lv_solid[l];
    lr.info = info[s];
    for (int k = 0; k < kSolidPar; k++) lr.par[k] = q[(size_t)s * kSolidStride + k];
    lr.mat = gr.mat_base + d->lv_mat[l];
    lr.dau_base = gr.pv_base + d->lv_dau_off[l];
    lr.dau_cnt = d->lv_dau_cnt[l];
    lr.vox = 0;
    lr.lclass = -1;
    bool want = d->lv_voxelize ? d->lv_voxelize[l] != 0 : true;
    if (want && d->lv_dau_cnt[l] >= 3) {
      std::vector<DauShape> db;
      for (int k = 0; k < d->lv_dau_cnt[l]; k++) {
        int p = d->lv_dau_off[l] + k;
        int ds = d->lv_solid[d->pv_lv[p]];
        DauShape sh;
        sh.box = place_solid(d->solid_type[ds], d->solid_par + 8 * ds, ext[ds], d->pv_rot + 9 * p,
                             d->pv_trans + 3 * p);
        for (int a = 0; a < 3; a++) {
          double pad = 1e-7 + 1e-12 * std::max(std::fabs(sh.box.lo[a]), std::fabs(sh.box.hi[a]));
          sh.box.lo[a] -= pad;
          sh.box.hi[a] += pad;
        }
        sh.info = info[ds];
        for (int i = 0; i < kSolidPar; i++) sh.q[i] = q[(size_t)ds * kSolidStride + i];
        for (int i = 0; i < 9; i++) sh.R[i] = d->pv_rot[9 * p + i];
        for (int i = 0; i < 3; i++) sh.t[i] = d->pv_trans[3 * p + i];
        db.push_back(sh);
      }
      VoxBuild vb = build_voxels(ext[d->lv_solid[l]], db, d->voxel_lists == 0);
      lr.vox = 1;
      lr.lclass = gr.n_class++;
      lr.node_base = (int)c->vox_node.size();
      for (int a = 0; a < 3; a++) {
        lr.n[a] = vb.n[a];
        lr.vlo[a] = vb.lo[a];
        lr.vw[a] = vb.w[a];
        lr.vinv[a] = vb.inv_w[a];
      }
      std::map<std::vector<uint16_t>, int> dedup;
      for (auto& nd : vb.nodes) {
        auto it = dedup.find(nd);
        int off;
        if (it == dedup.end()) {
          off = (int)c->vox_cand.size();
          c->vox_cand.insert(c->vox_cand.end(), nd.begin(), nd.end());
          dedup.emplace(nd, off);
        } else {
          off = it->second;
        }
        c->vox_node.push_back(int2{off, (int)nd.size()});
      }
      double mean = 0;
      for (auto& nd : vb.nodes) mean += (double)nd.size();
      mean /= std::max<size_t>(1, vb.nodes.size());
      lr.wide = mean >= kOrderMinCand ? 1 : 0;
      gr.any_wide = gr.any_wide || lr.wide;
    }
    c->lv_rec.push_back(lr);
  }
  // FP32 twins: mother parameters per LV, and per placement everything a
  // candidate test reads (bounding box rounded outward)
  for (int l = gr.lv_base; l < (int)c->lv_rec.size(); l++)
    for (int k = 0; k < kSolidPar; k++) c->lv_parf.push_back((float)c->lv_rec[l].par[k]);
  for (int p = gr.pv_base; p < (int)c->pv_rec.size(); p++) {
    const PRec& pr = c->pv_rec[p];
    const LRec& dl = c->lv_rec[pr.lv];
    PRecF pf;
    std::memset(&pf, 0, sizeof(pf));
    for (int a = 0; a < 3; a++) pf.t[a] = pr.m[9 + a];
    for (int k = 0; k < 9; k++) pf.r[k] = (float)pr.m[k];
    pf.kind = pr.kind;
    float bs = 0.f;
    for (int a = 0; a < 3; a++) {
      pf.lo[a] = round_down_f(pr.box_lo[a]);
      pf.hi[a] = round_up_f(pr.box_hi[a]);
      bs = std::max(bs, std::max(std::fabs(pf.lo[a]), std::fabs(pf.hi[a])));
    }
    pf.bscale = bs;
    pf.info = dl.info;
    float ss = 0.f;
    for (int k = 0; k < kSolidPar; k++) {
      pf.par[k] = (float)dl.par[k];
      ss = std::max(ss, std::fabs(pf.par[k]));
    }
    pf.sscale = ss;
    int ty = dl.info & 15;
    pf.sgrow = (ty == kTubs || ty == kCons)
                   ? 1.f + (float)std::max(std::fabs(dl.par[R_BO]), std::fabs(dl.par[R_BI]))
                   : 1.f;
    c->pvf.push_back(pf);
  }
  // touchables: breadth first from the world
  gr.h_parent.assign(nt, -1);
  gr.h_pv.assign(nt, -1);
  gr.h_lv.assign(nt, 0);
  gr.h_depth.assign(nt, 0);
  std::vector<int> slot(nt, 0), child(nt, 0);
  std::vector<long double> Rg((size_t)nt * 9), tg((size_t)nt * 3);
  gr.h_lv[0] = d->world_lv;
  for (int i = 0; i < 9; i++) Rg[i] = (i % 4 == 0) ? 1.0L : 0.0L;
  for (int i = 0; i < 3; i++) tg[i] = 0.0L;
  int n = 1;
  for (int i = 0; i < n; i++) {
    int l = gr.h_lv[i];
    child[i] = n;
    for (int k = 0; k < d->lv_dau_cnt[l]; k++) {
      int p = d->lv_dau_off[l] + k;
      gr.h_parent[n] = i;
      gr.h_pv[n] = p;
      gr.h_lv[n] = d->pv_lv[p];
      gr.h_depth[n] = gr.h_depth[i] + 1;
      slot[n] = k;
      const double* R = d->pv_rot + 9 * p;
      const double* t = d->pv_trans + 3 * p;
      // x_world = Rg_parent (R x + t) + tg_parent
      for (int a = 0; a < 3; a++) {
        for (int b = 0; b < 3; b++) {
          long double sum = 0;
          for (int m = 0; m < 3; m++) sum += Rg[(size_t)i * 9 + 3 * a + m] * (long double)R[3 * m + b];
          Rg[(size_t)n * 9 + 3 * a + b] = sum;
        }
        long double sum = tg[(size_t)i * 3 + a];
        for (int m = 0; m < 3; m++) sum += Rg[(size_t)i * 9 + 3 * a + m] * (long double)t[m];
        tg[(size_t)n * 3 + a] = sum;
      }
      n++;
    }
  }
  for (int i = 0; i < nt; i++) {
    bool ident = true;
    double M[9];
    for (int a = 0; a < 3; a++)
      for (int b = 0; b < 3; b++) {
        M[3 * a + b] = (double)Rg[(size_t)i * 9 + 3 * b + a];  // transpose
        if (M[3 * a + b] != (a == b ? 1.0 : 0.0)) ident = false;
      }
    c->t_xf.insert(c->t_xf.end(), M, M + 9);
    for (int a = 0; a < 3; a++) c->t_xf.push_back((double)tg[(size_t)i * 3 + a]);
    TRec tr;
    tr.lv = gr.lv_base + gr.h_lv[i];
    tr.parent = gr.h_parent[i] < 0 ? -1 : gr.t_base + gr.h_parent[i];
    tr.child_base = gr.t_base + child[i];
    tr.slot_kind = (slot[i] & 0xFFFF) | ((ident ? 0 : 1) << 16) | (std::min(gr.h_depth[i], 127) << 24);
    c->t_rec.push_back(tr);
  }
  c->geom_tbase.push_back(gr.t_base);
  int id = (int)c->geoms.size();
  c->geoms.push_back(std::move(gr));
  HIP_TRY(c, hipSetDevice(c->device), "hipSetDevice");
  hipError_t e = upload_all(c, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(c, e, "geometry upload");
  if (geom_id) *geom_id = id;
  if (n_touchables) *n_touchables = nt;
  return GNAV_OK;
}

gnav_status gnav_touchables(gnav_ctx* c, int32_t geom_id, int32_t* parent, int32_t* pv, int32_t* lv,
                            int32_t* depth) {
  gnav_status s = check_geom(c, geom_id);
  if (s) return s;
  const GeomRec& g = c->geoms[geom_id];
  for (int i = 0; i < g.n_t; i++) {
    if (parent) parent[i] = g.h_parent[i];
    if (pv) pv[i] = g.h_pv[i];
    if (lv) lv[i] = g.h_lv[i];
    if (depth) depth[i] = g.h_depth[i];
  }
  return GNAV_OK;
}

}  // extern "C"

namespace gnav {
// A network is being freed: unbind it from every geometry of the context.
void unbind_mlp(gnav_ctx* c, const gnav_mlp* mlp) {
  if (!c || !mlp) return;
  for (GeomRec& g : c->geoms)
    if (g.mlp == mlp) {
      g.mlp = nullptr;
      g.mlp_gen++;
    }
}
}  // namespace gnav

extern "C" {

gnav_status gnav_ordering_classes(gnav_ctx* c, int32_t geom_id, int32_t* n_class) {
  gnav_status s = check_geom(c, geom_id);
  if (s) return s;
  if (!n_class) return GNAV_EINVAL;
  *n_class = c->geoms[geom_id].n_class;
  return GNAV_OK;
}

gnav_status gnav_set_mlp(gnav_ctx* c, int32_t geom_id, gnav_mlp* mlp) {
  gnav_status s = check_geom(c, geom_id);
  if (s) return s;
  MlpView v;
  if (mlp && mlp_owner(mlp) != c) return fail(c, GNAV_EINVAL, "network belongs to another context");
  if (mlp && (!mlp_view(mlp, &v) || v.n_class != c->geoms[geom_id].n_class))
    return fail(c, GNAV_EINVAL, "network class count differs from the geometry's ordering classes");
  c->geoms[geom_id].mlp = mlp;
  c->geoms[geom_id].mlp_gen++;
  return GNAV_OK;
}

gnav_status gnav_touchable_offset(gnav_ctx* c, int32_t geom_id, int32_t* offset, int32_t* total) {
  gnav_status s = check_geom(c, geom_id);
  if (s) return s;
  if (offset) *offset = c->geoms[geom_id].t_base;
  if (total) *total = (int32_t)c->t_rec.size();
  return GNAV_OK;
}

gnav_status gnav_locate(gnav_ctx* c, int32_t geom_id, int64_t n, const double* pos, const double* dir,
                        int32_t* out, int32_t precision, void* stream) {
  gnav_status s = check_geom(c, geom_id);
  if (s) return s;
  if (n < 0 || (n > 0 && (!pos || !out))) return fail(c, GNAV_EINVAL, "bad locate arguments");
  if (precision < GNAV_PREC_FP64 || precision > GNAV_PREC_FP32) return fail(c, GNAV_EINVAL, "bad precision");
  // point-in-volume decisions are FP64 in every precision form
  int tb = c->geoms[geom_id].t_base;
  HIP_TRY(c, launch_locate(c->G, tb, tb, n, pos, dir, out, (hipStream_t)stream), "locate launch");
  return GNAV_OK;
}

gnav_status gnav_compute_step_ex(gnav_ctx* c, int32_t geom_id, int64_t n, const double* pos, const double* dir,
                                 const int32_t* touch, const double* max_step, int32_t precision, int32_t learned,
                                 const gnav_step_outputs* out, void* stream) {
  gnav_status s = check_geom(c, geom_id);
  if (s) return s;
  if (!out) return fail(c, GNAV_EINVAL, "null output description");
  if (n < 0 || (n > 0 && (!pos || !dir || !out->step_dev || !out->limiter_dev)))
    return fail(c, GNAV_EINVAL, "bad step arguments");
  if (precision < GNAV_PREC_FP64 || precision > GNAV_PREC_FP32) return fail(c, GNAV_EINVAL, "bad precision");
  if (learned < 0 || learned > 2) return fail(c, GNAV_EINVAL, "learned must be 0, 1 or 2");
  if (learned != 0 && precision != GNAV_PREC_FP64)
    return fail(c, GNAV_EINVAL, "candidate orders need FP64 distances");
  const GeomRec& gr = c->geoms[geom_id];
  StepArgs a{};
  a.G = c->G;
  a.W = a.tbase = gr.t_base;
  a.tcount = gr.n_t;
  a.n = n;
  a.pos = pos;
  a.dir = dir;
  a.touch = touch;
  a.max_step = max_step;
  a.step = out->step_dev;
  a.lim = out->limiter_dev;
  a.next = out->next_touchable_dev;
  a.saf = out->safety_dev;
  a.normal = out->normal_dev;
  a.normal_valid = out->normal_valid_dev;
  int order = learned;
  if (learned == 2) {
    if (!gr.mlp || !mlp_view(gr.mlp, &a.mlp) || a.mlp.n_class != gr.n_class)
      return fail(c, GNAV_ESTATE, "no network (or a class-count mismatch) for the learned order");
    // with no mother wide enough to order, the network would score nothing
    if (!gr.any_wide) order = 1;
  }
  HIP_TRY(c, launch_step(a, precision, order, (hipStream_t)stream), "step launch");
  return GNAV_OK;
}

gnav_status gnav_compute_step(gnav_ctx* c, int32_t geom_id, int64_t n, const double* pos, const double* dir,
                              const int32_t* touch, const double* max_step, double* step, int32_t* lim,
                              int32_t* next, int32_t precision, int32_t learned, void* stream) {
  gnav_step_outputs o{};
  o.step_dev = step;
  o.limiter_dev = lim;
  o.next_touchable_dev = next;
  return gnav_compute_step_ex(c, geom_id, n, pos, dir, touch, max_step, precision, learned, &o, stream);
}

gnav_status gnav_free_path(gnav_ctx* c, int32_t geom_id, int64_t n, const double* pos, const double* dir,
                           const double* life, double energy, double mu_mass, double* t_out, int32_t* nb_out,
                           void* stream) {
  gnav_status s = check_geom(c, geom_id);
  if (s) return s;
  if (n < 0 || (n > 0 && (!pos || !dir || !life || !t_out))) return fail(c, GNAV_EINVAL, "bad free-path arguments");
  if (!(mu_mass >= 0) || !std::isfinite(mu_mass)) return fail(c, GNAV_EINVAL, "bad mass attenuation");
  if (mu_mass == 0 && !(energy > 0 && std::isfinite(energy))) return fail(c, GNAV_EINVAL, "bad energy");
  int tb = c->geoms[geom_id].t_base;
  HIP_TRY(c, launch_free_path(c->G, tb, n, pos, dir, life, energy, mu_mass, t_out, nb_out, (hipStream_t)stream),
          "free-path launch");
  return GNAV_OK;
}

gnav_status gnav_compute_safety(gnav_ctx* c, int32_t geom_id, int64_t n, const double* pos,
                                const int32_t* touch, double* out, int32_t precision, void* stream) {
  gnav_status s = check_geom(c, geom_id);
  if (s) return s;
  if (n < 0 || (n > 0 && (!pos || !out))) return fail(c, GNAV_EINVAL, "bad safety arguments");
  if (precision < GNAV_PREC_FP64 || precision > GNAV_PREC_FP32) return fail(c, GNAV_EINVAL, "bad precision");
  int tb = c->geoms[geom_id].t_base;
  HIP_TRY(c, launch_safety(c->G, tb, tb, c->geoms[geom_id].n_t, n, pos, touch, out, precision,
                           (hipStream_t)stream),
          "safety launch");
  return GNAV_OK;
}

gnav_status gnav_tally_create(gnav_ctx* c, int32_t n_events, gnav_tally** out) {
  if (!c || !out || n_events < 0) return GNAV_EINVAL;
  *out = nullptr;
  if (c->geoms.empty()) return fail(c, GNAV_ESTATE, "no geometry uploaded");
  gnav_tally* t = new (std::nothrow) gnav_tally();
  if (!t) return fail(c, GNAV_ENOMEM, "tally");
  t->n_events = n_events;
  t->n_touch = (int)c->t_rec.size();
  hipError_t e;
  if ((e = t->edep_t.upload(nullptr, sizeof(double) * t->n_touch)) != hipSuccess ||
      (e = t->edep_ev.upload(nullptr, sizeof(double) * (size_t)n_events)) != hipSuccess ||
      (e = t->esc_ev.upload(nullptr, sizeof(double) * (size_t)n_events)) != hipSuccess ||
      (e = t->counters.upload(nullptr, sizeof(unsigned long long) * GNAV_NCOUNTERS)) != hipSuccess ||
      (e = hipStreamSynchronize(nullptr)) != hipSuccess) {
    delete t;
    return hip_fail(c, e, "tally allocation");
  }
  *out = t;
  return GNAV_OK;
}

gnav_status gnav_tally_reset(gnav_ctx* c, gnav_tally* t, void* stream) {
  if (!c || !t) return GNAV_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(c, zero_tally(t, st), "tally reset");
  return GNAV_OK;
}

gnav_status gnav_tally_free(gnav_ctx* c, gnav_tally* t) {
  if (!c) return GNAV_EINVAL;
  delete t;
  return GNAV_OK;
}

}  // extern "C"

namespace {

// Validate a batch and fill the launch description (may grow the
// pending-photon buffer, which synchronises the stream).
// Default track-pool slots per block (the fastest of 64 / 128 / 256 on the
// calorimeter and on the barrel).
constexpr int kDefaultBlock = 64;

// Default grid: two waves per SIMD are resident (eight per compute unit, so
// 2 * 256 / block blocks), and half as many again wait to take over from
// blocks that run out of work early; no more blocks than the batch fills.
int default_grid(const gnav_ctx* c, int block, long n) {
  long need = std::max<long>(1, (n + block - 1) / block);
  return (int)std::min<long>(need, (long)c->n_cu * 3 * (256 / block));
}

std::array<int, 4> tuning_key(const gnav_batch* b) {
  int lg = 0;
  while (lg < 62 && (1LL << (lg + 1)) <= b->n_primaries) lg++;
  return {b->geom_id, b->precision, b->order, lg};
}

// With `noalloc` the queue counter and pending photons live in the device's
// scratch array instead of the context's buffers, and nothing is allocated.
gnav_status prepare_transport(gnav_ctx* c, const gnav_batch* b, gnav_tally* t, hipStream_t stream,
                              TransportLaunch* out, bool noalloc = false) {
  if (!c || !b || !t) return GNAV_EINVAL;
  gnav_status s = check_geom(c, b->geom_id);
  if (s) return s;
  if (b->n_primaries < 0 || b->n_primaries > 0x7fffffffL) return fail(c, GNAV_EINVAL, "primary count out of range");
  if (b->n_primaries > 0 && (!b->event_dev || !b->prim_id_dev || !b->pos_dev || !b->dir_dev || !b->energy_dev))
    return fail(c, GNAV_EINVAL, "null primary array");
  if (t->n_touch != (int)c->t_rec.size())
    return fail(c, GNAV_ESTATE, "tally was created before the last geometry upload");
  if (b->precision < GNAV_PREC_FP64 || b->precision > GNAV_PREC_FP32)
    return fail(c, GNAV_EINVAL, "precision must be GNAV_PREC_FP64, _FP32_SCREENED or _FP32");
  if (b->precision != GNAV_PREC_FP64 && (b->order != 0 || b->record_dev))
    return fail(c, GNAV_EINVAL, "candidate orders and the crossing recorder need FP64 distances");
  if (b->log_dev && (b->log_capacity <= 0 || !b->log_n_dev || !b->log_fate_dev))
    return fail(c, GNAV_EINVAL, "log buffers incomplete");
  if (!b->log_dev && !b->digest_dev && (b->log_n_dev || b->log_fate_dev))
    return fail(c, GNAV_EINVAL, "log counts without a log or digests");
  if (!(b->e_cut >= 0)) return fail(c, GNAV_EINVAL, "bad energy cut");
  if (b->max_steps_per_track > GNAV_MAX_STEPS_PER_TRACK)
    return fail(c, GNAV_EINVAL, "max_steps_per_track above GNAV_MAX_STEPS_PER_TRACK");
  int grid_req = b->grid, chunk_req = b->chunk, sort_req = b->sort_period, block_req = b->block;
  if (b->tuned) {
    auto it = c->tuning.find(tuning_key(b));
    if (it != c->tuning.end()) {
      block_req = it->second.block;
      grid_req = it->second.grid;
      chunk_req = it->second.chunk;
      sort_req = it->second.sort_period;
    }
  }
  int block = block_req > 0 ? block_req : kDefaultBlock;
  if (block != 64 && block != 128 && block != 256)
    return fail(c, GNAV_EINVAL, "block must be 64, 128 or 256 (the track-pool slots of a block)");
  long need = (b->n_primaries + block - 1) / block;
  int grid = grid_req > 0 ? grid_req : default_grid(c, block, b->n_primaries);
  TransportLaunch& L = *out;
  L = TransportLaunch{};
  L.G = c->G;
  L.n = b->n_primaries;
  L.event = b->event_dev;
  L.prim_id = b->prim_id_dev;
  L.pos = b->pos_dev;
  L.dir = b->dir_dev;
  L.energy = b->energy_dev;
  L.event_geom = b->event_geom_dev;
  L.geom_default = b->geom_id;
  L.geom_tbase = c->d_geom_tbase.as<int>();
  L.n_geoms = (int)c->geoms.size();
  L.n_events = t->n_events;
  L.seed = b->seed;
  L.ecut = b->e_cut;
  L.max_steps = b->max_steps_per_track > 0 ? b->max_steps_per_track : 1000000;
  L.edep_t = t->edep_t.as<double>();
  L.edep_ev = t->edep_ev.as<double>();
  L.esc_ev = t->esc_ev.as<double>();
  L.counters = t->counters.as<unsigned long long>();
  if (noalloc) {
    if ((long)grid * block > GNAV_NOALLOC_MAX_SLOTS)
      return fail(c, GNAV_EINVAL, "grid * block = " + std::to_string((long)grid * block) +
                                      " track slots, above GNAV_NOALLOC_MAX_SLOTS = " +
                                      std::to_string(GNAV_NOALLOC_MAX_SLOTS) + " (pass a smaller grid)");
    if (!c->scratch) return fail(c, GNAV_ESTATE, "no scratch address for this device");
    L.queue = reinterpret_cast<unsigned long long*>(c->scratch);
    L.pend = reinterpret_cast<double*>(static_cast<char*>(c->scratch) + kNoallocQueueBytes);
  } else {
    L.queue = c->d_queue.as<unsigned long long>();
    // per-slot storage for the second annihilation photon of a pair conversion
    size_t pend_bytes = (size_t)grid * block * 6 * sizeof(double);
    if (c->d_pend.bytes < pend_bytes) {
      HIP_TRY(c, hipDeviceSynchronize(), "synchronize");
      HIP_TRY(c, c->d_pend.upload(nullptr, pend_bytes, stream), "pending-photon buffer");
      HIP_TRY(c, hipStreamSynchronize(stream), "synchronize");
      c->pend_gen++;
    }
    L.pend = c->d_pend.as<double>();
    const int keys = b->event_geom_dev ? kClaimClasses * (int)c->geoms.size() : kClaimClasses;
    if (!b->keep_order && b->n_primaries > 0 && keys <= kClaimMaxKeys) {
      // the key counts and cursors, then the primaries copied in claim order
      size_t claim_bytes = 2 * kClaimMaxKeys * sizeof(unsigned) + (size_t)b->n_primaries * sizeof(ClaimRec);
      if (c->d_claim.bytes < claim_bytes) {
        HIP_TRY(c, hipDeviceSynchronize(), "synchronize");
        HIP_TRY(c, c->d_claim.upload(nullptr, claim_bytes, stream), "claim-order buffer");
        HIP_TRY(c, hipStreamSynchronize(stream), "synchronize");
        c->pend_gen++;
      }
      L.claim_cnt = c->d_claim.as<unsigned>();
      L.claim = reinterpret_cast<ClaimRec*>(c->d_claim.as<unsigned>() + 2 * kClaimMaxKeys);
      L.claim_keys = keys;
    }
  }
  L.count = b->count_work != 0;
  if (b->order < 0 || b->order > 2) return fail(c, GNAV_EINVAL, "order must be 0, 1 or 2");
  // With no mother wide enough for ordered walks the learned order scores
  // nothing and walks like the bound order; launch that instantiation.
  L.order = (b->order == 2 && !c->geoms[b->geom_id].any_wide) ? 1 : b->order;
  L.prec = b->precision;
  if (chunk_req < 0 || chunk_req > (1 << 24)) return fail(c, GNAV_EINVAL, "chunk out of range");
  if (sort_req < 0) return fail(c, GNAV_EINVAL, "negative sort period");
  L.chunk = chunk_req;
  L.sort_period = sort_req;
  L.G_n_lv = std::max(1, (int)c->lv_rec.size());
  if (b->order == 2) {
    const GeomRec& gr = c->geoms[b->geom_id];
    if (b->event_geom_dev) return fail(c, GNAV_EUNSUPPORTED, "the learned order needs a single geometry");
    if (!gr.mlp || !mlp_view(gr.mlp, &L.mlp) || L.mlp.n_class != gr.n_class)
      return fail(c, GNAV_ESTATE, "no network (or a class-count mismatch) for the learned order");
  }
  if (b->record_dev && (b->record_capacity <= 0 || !b->record_count_dev))
    return fail(c, GNAV_EINVAL, "recorder buffers incomplete");
  L.rec = b->record_dev;
  L.rec_cap = b->record_dev ? b->record_capacity : 0;
  L.rec_count = reinterpret_cast<unsigned long long*>(b->record_count_dev);
  L.log = b->log_dev;
  L.digest = b->digest_dev;
  L.log_cap = b->log_dev ? b->log_capacity : 0;
  L.log_n = b->log_n_dev;
  L.log_fate = b->log_fate_dev;
  L.block = block;
  L.grid = grid;
  // a batch with per-event geometries can reach every resident geometry
  L.axis_boxes = b->event_geom_dev ? std::all_of(c->geoms.begin(), c->geoms.end(),
                                                 [](const GeomRec& g) { return g.axis_boxes; })
                                   : c->geoms[b->geom_id].axis_boxes;
  L.spheres = b->event_geom_dev ? std::any_of(c->geoms.begin(), c->geoms.end(),
                                              [](const GeomRec& g) { return g.spheres; })
                                : c->geoms[b->geom_id].spheres;
  return GNAV_OK;
}

}  // namespace

struct gnav_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // what the captured kernels hold, checked before every replay
  const gnav_ctx* ctx = nullptr;
  uint64_t tables_gen = 0, pend_gen = 0, mlp_gen = 0;
  int geom_id = -1;
  bool uses_mlp = false;
};

namespace {

// Order a launch of context c on `stream` after the context's previous
// launch when that one went to another stream (launches share the work
// queue and the pending-photon buffer), then remember this one.  A stream
// under capture is left alone: a captured launch is ordered when the graph is
// replayed (gnav_graph_launch applies the same rule).
hipError_t order_before(gnav_ctx* c, hipStream_t stream) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  hipError_t e = hipStreamIsCapturing(stream, &cs);
  if (e != hipSuccess) return e;
  if (cs != hipStreamCaptureStatusNone) return hipSuccess;
  if (c->launched && stream != c->last_stream) {
    e = hipStreamWaitEvent(stream, c->last_launch, 0);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t order_after(gnav_ctx* c, hipStream_t stream) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  hipError_t e = hipStreamIsCapturing(stream, &cs);
  if (e != hipSuccess) return e;
  if (cs != hipStreamCaptureStatusNone) return hipSuccess;
  e = hipEventRecord(c->last_launch, stream);
  if (e != hipSuccess) return e;
  c->last_stream = stream;
  c->launched = true;
  return hipSuccess;
}

}  // namespace

extern "C" {

gnav_status gnav_transport_batch(gnav_ctx* c, const gnav_batch* b, gnav_tally* t, void* stream) {
  TransportLaunch L;
  gnav_status s = prepare_transport(c, b, t, (hipStream_t)stream, &L);
  if (s) return s;
  HIP_TRY(c, order_before(c, (hipStream_t)stream), "stream ordering");
  HIP_TRY(c, launch_transport(L, (hipStream_t)stream), "transport launch");
  HIP_TRY(c, order_after(c, (hipStream_t)stream), "stream ordering");
  return GNAV_OK;
}

gnav_status gnav_transport_batch_noalloc(gnav_ctx* c, const gnav_batch* b, gnav_tally* t, void* stream) {
  TransportLaunch L;
  gnav_status s = prepare_transport(c, b, t, (hipStream_t)stream, &L, true);
  if (s) return s;
  HIP_TRY(c, order_before(c, (hipStream_t)stream), "stream ordering");
  HIP_TRY(c, launch_transport(L, (hipStream_t)stream), "transport launch");
  HIP_TRY(c, order_after(c, (hipStream_t)stream), "stream ordering");
  return GNAV_OK;
}

namespace {

// Median kernel time (ms) of `trials` runs of one launch setting, each on a
// freshly zeroed tally.
gnav_status time_setting(gnav_ctx* c, const gnav_batch& b, gnav_tally* t, hipStream_t st, int trials,
                         float* ms_out) {
  TransportLaunch L;
  gnav_status s = prepare_transport(c, &b, t, st, &L);
  if (s) return s;
  hipEvent_t e0, e1;
  HIP_TRY(c, hipEventCreate(&e0), "event");
  hipError_t e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_fail(c, e, "event");
  }
  std::vector<float> ms;
  for (int r = 0; r <= trials && e == hipSuccess; r++) {  // r = 0 warms up
    if ((s = gnav_tally_reset(c, t, st))) break;
    if ((e = hipEventRecord(e0, st)) != hipSuccess) break;
    if ((e = launch_transport(L, st)) != hipSuccess) break;
    if ((e = hipEventRecord(e1, st)) != hipSuccess) break;
    if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
    float v = 0;
    if ((e = hipEventElapsedTime(&v, e0, e1)) != hipSuccess) break;
    if (r > 0) ms.push_back(v);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s) return s;
  if (e != hipSuccess) return hip_fail(c, e, "autotune run");
  std::sort(ms.begin(), ms.end());
  *ms_out = ms[ms.size() / 2];
  return GNAV_OK;
}

}  // namespace

gnav_status gnav_autotune(gnav_ctx* c, const gnav_batch* batch, gnav_tally* t, int32_t trials, void* stream,
                          gnav_tuning* out) {
  if (!c || !batch || !t) return GNAV_EINVAL;
  if (trials < 1 || trials > 100) return fail(c, GNAV_EINVAL, "trials must be 1..100");
  if (batch->log_dev || batch->digest_dev || batch->record_dev)
    return fail(c, GNAV_EINVAL, "tune without the per-track log or the recorder");
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(c, order_before(c, st), "stream ordering");
  gnav_batch b = *batch;
  b.tuned = 0;
  // coordinate descent: block (pool size) with its default grid, then grid,
  // then chunk, then sort period
  gnav_tuning best{kDefaultBlock, default_grid(c, kDefaultBlock, b.n_primaries), 0, 0, 0.f};
  b.block = best.block;
  b.grid = best.grid;
  b.chunk = 0;
  b.sort_period = 0;
  gnav_status s = time_setting(c, b, t, st, trials, &best.ms);
  if (s) return s;
  auto consider = [&](gnav_batch cand) -> gnav_status {
    float ms = 0;
    gnav_status r = time_setting(c, cand, t, st, trials, &ms);
    if (r) return r;
    if (ms < best.ms) best = gnav_tuning{cand.block, cand.grid, cand.chunk, cand.sort_period, ms};
    return GNAV_OK;
  };
  for (int bl : {256, 128, 64}) {
    if (bl == kDefaultBlock) continue;
    gnav_batch cand = b;
    cand.block = bl;
    cand.grid = default_grid(c, bl, b.n_primaries);
    if ((s = consider(cand))) return s;
  }
  {
    const long need = std::max<long>(1, (b.n_primaries + best.block - 1) / best.block);
    const long resident = (long)c->n_cu * 2 * (256 / best.block);  // blocks resident at once
    for (long g : {resident / 2, resident, resident * 2, resident * 3}) {
      const int gg = (int)std::min<long>(need, std::max<long>(1, g));
      if (gg == best.grid) continue;
      gnav_batch cand = b;
      cand.block = best.block;
      cand.grid = gg;
      if ((s = consider(cand))) return s;
    }
  }
  for (int ch : {256, 1024, 4096}) {
    gnav_batch cand = b;
    cand.block = best.block;
    cand.grid = best.grid;
    cand.chunk = ch;
    if ((s = consider(cand))) return s;
  }
  for (int sp : {1, 4, 16}) {
    gnav_batch cand = b;
    cand.block = best.block;
    cand.grid = best.grid;
    cand.chunk = best.chunk;
    cand.sort_period = sp;
    if ((s = consider(cand))) return s;
  }
  if ((s = gnav_tally_reset(c, t, st))) return s;
  HIP_TRY(c, order_after(c, st), "stream ordering");
  HIP_TRY(c, hipStreamSynchronize(st), "synchronize");
  c->tuning[tuning_key(&b)] = best;
  if (out) *out = best;
  return GNAV_OK;
}

gnav_status gnav_graph_create(gnav_ctx* c, const gnav_batch* b, gnav_tally* t, void* stream, gnav_graph** out) {
  if (!out) return GNAV_EINVAL;
  *out = nullptr;
  hipStream_t st = (hipStream_t)stream;
  TransportLaunch L;
  gnav_status s = prepare_transport(c, b, t, st, &L);
  if (s) return s;
  HIP_TRY(c, hipStreamSynchronize(st), "synchronize");
  gnav_graph* g = new (std::nothrow) gnav_graph();
  if (!g) return fail(c, GNAV_ENOMEM, "graph");
  hipStream_t cap;
  hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete g;
    return hip_fail(c, e, "capture stream");
  }
  e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    hipError_t e1 = zero_tally(t, cap);
    hipError_t e2 = launch_transport(L, cap);
    hipError_t ee = hipStreamEndCapture(cap, &g->graph);
    e = e1 != hipSuccess ? e1 : e2 != hipSuccess ? e2 : ee;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  g->ctx = c;
  g->tables_gen = c->tables_gen;
  g->pend_gen = c->pend_gen;
  g->geom_id = b->geom_id;
  g->uses_mlp = L.order == kOrderLearned;
  g->mlp_gen = c->geoms[b->geom_id].mlp_gen;
  (void)hipStreamDestroy(cap);
  if (e != hipSuccess) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    return hip_fail(c, e, "graph capture");
  }
  *out = g;
  return GNAV_OK;
}

gnav_status gnav_graph_launch(gnav_ctx* c, gnav_graph* g, void* stream) {
  if (!c || !g) return GNAV_EINVAL;
  if (g->ctx != c) return fail(c, GNAV_EINVAL, "graph belongs to another context");
  if (g->tables_gen != c->tables_gen)
    return fail(c, GNAV_ESTATE, "geometry tables were reallocated after the capture (capture again)");
  if (g->pend_gen != c->pend_gen)
    return fail(c, GNAV_ESTATE, "launch buffers (pending photons, claim order) were reallocated after the capture "
                                "(capture again)");
  if (g->uses_mlp && g->mlp_gen != c->geoms[g->geom_id].mlp_gen)
    return fail(c, GNAV_ESTATE, "network binding changed after the capture (capture again)");
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(c, order_before(c, st), "stream ordering");
  HIP_TRY(c, hipGraphLaunch(g->exec, st), "graph launch");
  HIP_TRY(c, order_after(c, st), "stream ordering");
  return GNAV_OK;
}

gnav_status gnav_graph_free(gnav_ctx* c, gnav_graph* g) {
  if (!c) return GNAV_EINVAL;
  if (g) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
  }
  return GNAV_OK;
}

gnav_status gnav_read_tallies(gnav_ctx* c, const gnav_tally* t, double* edep_t, double* edep_ev,
                              double* esc_ev, uint64_t* counters, void* stream) {
  if (!c || !t) return GNAV_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(c, hipStreamSynchronize(st), "synchronize");
  if (edep_t) HIP_TRY(c, hipMemcpy(edep_t, t->edep_t.p, sizeof(double) * t->n_touch, hipMemcpyDeviceToHost), "read");
  if (edep_ev)
    HIP_TRY(c, hipMemcpy(edep_ev, t->edep_ev.p, sizeof(double) * t->n_events, hipMemcpyDeviceToHost), "read");
  if (esc_ev)
    HIP_TRY(c, hipMemcpy(esc_ev, t->esc_ev.p, sizeof(double) * t->n_events, hipMemcpyDeviceToHost), "read");
  if (counters)
    HIP_TRY(c, hipMemcpy(counters, t->counters.p, sizeof(uint64_t) * GNAV_NCOUNTERS, hipMemcpyDeviceToHost),
            "read");
  return GNAV_OK;
}

}  // extern "C"

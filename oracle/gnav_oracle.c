/*
 * gnav_oracle.c -- plain, slow CPU oracle for Geant4-style gamma navigation.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg do.  It shares no code, header, table or constant generator
 * with the GPU path.
 *
 * What it computes (Seiskari, Kommeri, Niemi, "GPU in Physics Computation:
 * Case Geant4 Navigation"):
 *   - the free-path sampling of Sec. 3.1, Alg. 1 and Eqs. 1-8: an Exp(1)
 *     optical depth Y = -log W, spent piecewise along the ray as
 *     S_j = S_{j-1} + (t_j - t_{j-1}) mu_j, interaction at
 *     T = t_{j-1} + (Y - S_{j-1}) / mu_j;
 *   - the two navigation queries of Sec. 3.2 (which volumes contain a point;
 *     where the ray next crosses a boundary), answered by brute force over
 *     every daughter of the current mother: no voxels, no caching (an
 *     optional cell-grid mode, og_set_voxels, gives the same answers faster
 *     and serves only as a CPU timing baseline);
 *   - a gamma transport loop that repeats Alg. 1 after every interaction
 *     (photoelectric, Klein-Nishina Compton, Bethe-Heitler pair), with energy
 *     tallies per touchable and per event.
 * The paper does not specify solids, tolerances, cross sections or the random
 * stream; the rules used for those are stated next to each function.
 *
 * Units: mm, MeV, rad; densities g/cm3; cross sections cm2 (converted to
 * 1/mm in the attenuation tables).  Parity status: pinned (see tests) except
 * the whole-transport physics against real data, which the paper does not
 * print ("parity unpinned" for that comparison).
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no fast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OG_BOX 0
#define OG_TUBS 1
#define OG_CONS 2
#define OG_ORB 3
#define OG_TRD 4
#define OG_SPHERE 5

#define OG_IN 1
#define OG_SURF 0
#define OG_OUT -1

/* Surface tolerance: a point within half of this of a surface is on it. */
static const double kTol = 1e-9;
static const double kHalf = 0.5e-9;
static const double kInf = INFINITY;

/* Physical constants (CODATA 2018). */
static const double kMe = 0.51099895;            /* electron rest energy, MeV */
static const long double kReL = 2.8179403262e-13L; /* classical electron radius, cm */
static const long double kNaL = 6.02214076e23L;    /* Avogadro, 1/mol */
static const long double kAlphaL = 1.0L / 137.035999084L;
static const long double kPiL = 3.141592653589793238462643383279502884L;
/* Photoelectric scale: sigma_pe = K Z^4 / E^3 with K = 4.0e-8 barn MeV^3. */
static const long double kPeK = 4.0e-32L;

/* Cross-section grid: 257 log-spaced nodes from 1 keV to 100 MeV. */
#define OG_NNODE 257

/* Transport limits. */
#define OG_ZERO_PUSH 10
#define OG_ZERO_KILL 25
#define OG_MAX_COMPTON_TRIALS 1000

/* Log limiter codes. */
#define OG_LIM_MOTHER -1
#define OG_LIM_PE -2
#define OG_LIM_COMPTON -3
#define OG_LIM_PAIR -4

/* Track fates. */
#define OG_FATE_ABSORBED 1
#define OG_FATE_ESCAPED 2
#define OG_FATE_CUTOFF 3
#define OG_FATE_STUCK 4
#define OG_FATE_TRUNCATED 5
#define OG_FATE_PAIR 6

/* Counter slots (same meaning as the library's read_tallies counters). */
enum {
  OG_C_STEPS = 0, OG_C_PE, OG_C_COMPTON, OG_C_PAIR, OG_C_CROSSINGS, OG_C_ESCAPED,
  OG_C_CUTOFF, OG_C_PUSHES, OG_C_STUCK, OG_C_TRUNCATED, OG_C_TRACKS, OG_NCOUNTERS
};

/* ------------------------------------------------------------------------ */
/* Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).        */
/* ------------------------------------------------------------------------ */

void og_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; r++) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

/* Draw number `draw` of track (event, key): counter {draw/2, key, event, 0},
 * key {seed low, seed high}; two 32-bit words make one 53-bit mantissa and
 * W = (m + 1) 2^-53 lies in (0, 1] as Alg. 1 step 1 requires. */
double og_uniform(uint64_t seed, uint32_t event, uint32_t key, uint32_t draw) {
  uint32_t ctr[4] = {draw >> 1, key, event, 0u};
  uint32_t k[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t o[4];
  og_philox4x32_10(ctr, k, o);
  uint32_t lo = o[2 * (draw & 1u)], hi = o[2 * (draw & 1u) + 1];
  uint64_t m = ((((uint64_t)hi) << 32) | (uint64_t)lo) >> 11;
  return (double)(m + 1u) * 0x1p-53;
}

typedef struct {
  uint64_t seed;
  uint32_t event, key, draw;
} og_stream;

static double og_next(og_stream* s) {
  double u = og_uniform(s->seed, s->event, s->key, s->draw);
  s->draw++;
  return u;
}

/* ------------------------------------------------------------------------ */
/* Cross sections per atom (cm2), in extended precision.                    */
/* ------------------------------------------------------------------------ */

/* Klein-Nishina total cross section per electron; k = E / (m_e c^2). */
long double og_kn_per_electron(long double k) {
  long double l = log1pl(2.0L * k);
  long double a = (1.0L + k) / (k * k) * (2.0L * (1.0L + k) / (1.0L + 2.0L * k) - l / k);
  long double b = l / (2.0L * k);
  long double c = (1.0L + 3.0L * k) / ((1.0L + 2.0L * k) * (1.0L + 2.0L * k));
  return 2.0L * kPiL * kReL * kReL * (a + b - c);
}

/* sigma per atom for photoelectric, Compton (Z electrons) and pair. */
void og_sigma_atom(int Z, double E, double out[3]) {
  long double e = (long double)E;
  long double z = (long double)Z;
  long double k = e / (long double)kMe;
  out[0] = (double)(kPeK * z * z * z * z / (e * e * e));
  out[1] = (double)(z * og_kn_per_electron(k));
  long double pair = 0.0L;
  if (k > 2.0L) {
    long double r = (k - 2.0L) / k;
    long double f_thr = 2.0L * kPiL / 3.0L * r * r * r;
    long double f_bh = 28.0L / 9.0L * logl(2.0L * k) - 218.0L / 27.0L;
    long double f_cs = 28.0L / 9.0L * logl(183.0L * powl(z, -1.0L / 3.0L)) - 2.0L / 27.0L;
    long double f = f_bh > f_thr ? f_bh : f_thr;
    if (f_cs < f) f = f_cs;
    pair = kAlphaL * kReL * kReL * z * z * f;
  }
  out[2] = (double)pair;
}

/* ------------------------------------------------------------------------ */
/* Solids.  Each solid is an intersection of components (outer and inner     */
/* radial surface, z slab, phi wedge); a signed value per component is       */
/* negative inside.  The solid's value d is the maximum over components:     */
/* d < -tol/2 inside, d > tol/2 outside, otherwise on the surface.           */
/* ------------------------------------------------------------------------ */

typedef struct {
  int type;
  double par[8];
  /* radial surfaces r(z) = A + B z, perpendicular factor c = 1/sqrt(1+B^2) */
  double Ao, Bo, co, Ai, Bi, ci, dz;
  int has_inner, has_phi;
  double ns[2], ne[2]; /* outward normals of the start and end phi planes */
  /* trapezoid: the six face planes n . p = h (n unit, outward): +x, -x, +y, -y, +z, -z */
  double pn[6][3], ph[6];
  /* sphere section: radii, and the two theta bounds as cone surfaces rho = B z
   * (B = tan theta, perpendicular factor c = |cos theta|) or the plane z = 0 */
  double srmin, srmax;
  int tkind[2];
  double tB[2], tc[2];
} og_solid;

/* Kinds of a sphere section's theta bound: none; a cone whose solid inside
 * (rho <= B z on the sheet B z >= 0) is the allowed region (outer); a cone
 * whose outside is (inner); the half-space z <= 0 or z >= 0 (theta = pi/2). */
enum { T_NONE = 0, T_OUTER, T_INNER, T_ZLE, T_ZGE };
/* sphere component slots */
enum { S_RO = 0, S_RI, S_PA, S_PB, S_T1, S_T2, S_N };

/* component slots */
enum { K_RO = 0, K_RI, K_Z, K_PA, K_PB, K_N };

static int solid_init(og_solid* s, int type, const double* par) {
  memset(s, 0, sizeof(*s));
  s->type = type;
  memcpy(s->par, par, 8 * sizeof(double));
  if (type == OG_BOX) {
    return (par[0] > 0 && par[1] > 0 && par[2] > 0) ? 0 : -1;
  }
  if (type == OG_ORB) {
    return par[0] > 0 ? 0 : -1;
  }
  if (type == OG_TRD) {
    /* half lengths dx1, dx2 (x at z = -dz, +dz), dy1, dy2, half length dz: the
     * x faces are the planes |x| = ax + bx z, ax = (dx1 + dx2) / 2,
     * bx = (dx2 - dx1) / (2 dz), likewise y */
    double dx1 = par[0], dx2 = par[1], dy1 = par[2], dy2 = par[3], dz = par[4];
    if (!(dx1 > 0 && dx2 > 0 && dy1 > 0 && dy2 > 0 && dz > 0)) return -1;
    double a[2] = {0.5 * (dx1 + dx2), 0.5 * (dy1 + dy2)};
    double b[2] = {(dx2 - dx1) / (2.0 * dz), (dy2 - dy1) / (2.0 * dz)};
    for (int ax = 0; ax < 2; ax++) {
      double c = 1.0 / sqrt(1.0 + b[ax] * b[ax]);
      for (int sg = 0; sg < 2; sg++) {
        double* n = s->pn[2 * ax + sg];
        n[0] = n[1] = n[2] = 0.0;
        n[ax] = (sg == 0 ? 1.0 : -1.0) * c;
        n[2] = -b[ax] * c;
        s->ph[2 * ax + sg] = a[ax] * c;
      }
    }
    s->pn[4][0] = s->pn[4][1] = s->pn[5][0] = s->pn[5][1] = 0.0;
    s->pn[4][2] = 1.0;
    s->pn[5][2] = -1.0;
    s->ph[4] = s->ph[5] = dz;
    s->dz = dz;
    return 0;
  }
  if (type == OG_SPHERE) {
    /* rmin, rmax, sphi, dphi, stheta, dtheta */
    double rmin = par[0], rmax = par[1], sphi = par[2], dphi = par[3], st = par[4], dt = par[5];
    const double twopi = 2.0 * M_PI;
    if (!(rmin >= 0) || !(rmax > rmin) || (rmin > 0 && rmin < kTol)) return -1;
    if (!(dphi > 0) || dphi > twopi || (dphi < twopi && dphi > M_PI)) return -1;
    if (!(st >= 0) || !(dt > 0) || st + dt > M_PI * (1.0 + 1e-15)) return -1;
    s->srmin = rmin;
    s->srmax = rmax;
    s->has_inner = rmin > 0;
    s->has_phi = dphi < twopi;
    if (s->has_phi) {
      double ephi = sphi + dphi;
      s->ns[0] = sin(sphi);
      s->ns[1] = -cos(sphi);
      s->ne[0] = -sin(ephi);
      s->ne[1] = cos(ephi);
    }
    const double th[2] = {st, st + dt};
    for (int j = 0; j < 2; j++) {
      /* lower bound theta >= th[0]: a bound only above 0; upper bound
       * theta <= th[1]: only below pi */
      int present = j == 0 ? th[0] > 0 : th[1] < M_PI;
      s->tkind[j] = T_NONE;
      if (!present) continue;
      if (th[j] == 0.5 * M_PI) {
        s->tkind[j] = j == 0 ? T_ZLE : T_ZGE;
        continue;
      }
      s->tB[j] = tan(th[j]);
      s->tc[j] = 1.0 / sqrt(1.0 + s->tB[j] * s->tB[j]);
      int lower_half = th[j] > 0.5 * M_PI;
      /* theta >= th below the equator and theta <= th above it keep the
       * outside of the cone; the other two its inside */
      s->tkind[j] = (j == 0) != lower_half ? T_INNER : T_OUTER;
    }
    return 0;
  }
  double rmin1, rmax1, rmin2, rmax2, dz, sphi, dphi;
  if (type == OG_TUBS) {
    rmin1 = rmin2 = par[0];
    rmax1 = rmax2 = par[1];
    dz = par[2];
    sphi = par[3];
    dphi = par[4];
  } else if (type == OG_CONS) {
    rmin1 = par[0];
    rmax1 = par[1];
    rmin2 = par[2];
    rmax2 = par[3];
    dz = par[4];
    sphi = par[5];
    dphi = par[6];
  } else {
    return -1;
  }
  if (!(dz > 0) || !(rmin1 >= 0) || !(rmin2 >= 0) || !(rmax1 > rmin1) || !(rmax2 > rmin2)) return -1;
  if ((rmin1 > 0 && rmin1 < kTol) || (rmin2 > 0 && rmin2 < kTol)) return -1;
  const double twopi = 2.0 * M_PI;
  if (!(dphi > 0)) return -1;
  if (dphi < twopi && dphi > M_PI) return -1; /* wedges wider than pi are not supported */
  if (dphi > twopi) return -1;
  s->dz = dz;
  s->Ao = 0.5 * (rmax1 + rmax2);
  s->Bo = (rmax2 - rmax1) / (2.0 * dz);
  s->co = 1.0 / sqrt(1.0 + s->Bo * s->Bo);
  s->Ai = 0.5 * (rmin1 + rmin2);
  s->Bi = (rmin2 - rmin1) / (2.0 * dz);
  s->ci = 1.0 / sqrt(1.0 + s->Bi * s->Bi);
  s->has_inner = (rmin1 > 0 || rmin2 > 0);
  s->has_phi = dphi < twopi;
  if (s->has_phi) {
    double ephi = sphi + dphi;
    s->ns[0] = sin(sphi);
    s->ns[1] = -cos(sphi);
    s->ne[0] = -sin(ephi);
    s->ne[1] = cos(ephi);
  }
  return 0;
}

static double max2(double a, double b) { return a > b ? a : b; }
static double min2(double a, double b) { return a < b ? a : b; }

/* Decision margins (for telling a rounding-edge flip from a real difference
 * when a track's history differs from another implementation's).  Each
 * decision taken while transporting a track -- a comparison of a with b --
 * notes |a - b| / scale; the smallest since the track's previous step record
 * is stored with the next record.  scale is the magnitude that sets the
 * rounding of the compared values: the geometry's coordinate extent for
 * lengths (og_scale), 1 for directions and uniform numbers, the operand
 * itself for attenuations and energies.  Off unless margins are requested. */
static int og_margin_on = 0;
static double og_margin = INFINITY;
static double og_scale = 1.0;

/* Comparisons that cannot change a result are not noted: a direction
 * component against zero (a slab or plane parallel to the ray gives the same
 * distances as a nearly parallel one) and the branch of the quadratic formula
 * (both branches give the same roots). */
static void note(double a, double b, double scale) {
  if (!og_margin_on) return;
  double m = fabs(a - b) / scale;
  if (a == b) m = 0.0; /* also inf == inf */
  if (m < og_margin) og_margin = m;
}
#define NOTE_LEN(a, b) note((a), (b), og_scale)

/* Component values of a radial solid (tubs or cons) at p. */
static void rad_comps(const og_solid* s, const double* p, double k[K_N]) {
  double rho = sqrt(p[0] * p[0] + p[1] * p[1]);
  k[K_RO] = (rho - (s->Ao + s->Bo * p[2])) * s->co;
  k[K_RI] = s->has_inner ? ((s->Ai + s->Bi * p[2]) - rho) * s->ci : -kInf;
  k[K_Z] = fabs(p[2]) - s->dz;
  if (s->has_phi) {
    k[K_PA] = p[0] * s->ns[0] + p[1] * s->ns[1];
    k[K_PB] = p[0] * s->ne[0] + p[1] * s->ne[1];
  } else {
    k[K_PA] = -kInf;
    k[K_PB] = -kInf;
  }
}

/* Signed distance of p from face plane i of a trapezoid (negative inside). */
static double trd_plane(const og_solid* s, int i, const double* p) {
  return s->pn[i][0] * p[0] + s->pn[i][1] * p[1] + s->pn[i][2] * p[2] - s->ph[i];
}

static double trd_dot(const og_solid* s, int i, const double* v) {
  return s->pn[i][0] * v[0] + s->pn[i][1] * v[1] + s->pn[i][2] * v[2];
}

/* Component values of a sphere section at p (-inf for absent faces). */
static void sph_comps(const og_solid* s, const double* p, double k[S_N]) {
  double r = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
  double rho = sqrt(p[0] * p[0] + p[1] * p[1]);
  k[S_RO] = r - s->srmax;
  k[S_RI] = s->has_inner ? s->srmin - r : -kInf;
  if (s->has_phi) {
    k[S_PA] = p[0] * s->ns[0] + p[1] * s->ns[1];
    k[S_PB] = p[0] * s->ne[0] + p[1] * s->ne[1];
  } else {
    k[S_PA] = -kInf;
    k[S_PB] = -kInf;
  }
  for (int j = 0; j < 2; j++) {
    double* kj = &k[S_T1 + j];
    switch (s->tkind[j]) {
      case T_OUTER: *kj = (rho - (0.0 + s->tB[j] * p[2])) * s->tc[j]; break;
      case T_INNER: *kj = ((0.0 + s->tB[j] * p[2]) - rho) * s->tc[j]; break;
      case T_ZLE: *kj = p[2]; break;
      case T_ZGE: *kj = -p[2]; break;
      default: *kj = -kInf; break;
    }
  }
}

/* Gradient (unnormalised where noted in sph_normal) dot v of sphere component i. */
static double sph_comp_dot(const og_solid* s, int i, const double* p, const double* v) {
  double r = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
  double rho = sqrt(p[0] * p[0] + p[1] * p[1]);
  double pv = p[0] * v[0] + p[1] * v[1] + p[2] * v[2];
  double rv = rho > 0 ? (p[0] * v[0] + p[1] * v[1]) / rho : 0.0;
  switch (i) {
    case S_RO: return r > 0 ? pv / r : 0.0;
    case S_RI: return r > 0 ? -pv / r : 0.0;
    case S_PA: return v[0] * s->ns[0] + v[1] * s->ns[1];
    case S_PB: return v[0] * s->ne[0] + v[1] * s->ne[1];
    default: {
      int j = i - S_T1;
      switch (s->tkind[j]) {
        case T_OUTER: return rv - s->tB[j] * v[2];
        case T_INNER: return -rv + s->tB[j] * v[2];
        case T_ZLE: return v[2];
        case T_ZGE: return -v[2];
        default: return 0.0;
      }
    }
  }
}

/* The solid's signed value d(p). */
double og_solid_d(const og_solid* s, const double* p) {
  if (s->type == OG_BOX) {
    double a = fabs(p[0]) - s->par[0];
    double b = fabs(p[1]) - s->par[1];
    double c = fabs(p[2]) - s->par[2];
    return max2(max2(a, b), c);
  }
  if (s->type == OG_ORB) {
    return sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]) - s->par[0];
  }
  if (s->type == OG_TRD) {
    double d = -kInf;
    for (int i = 0; i < 6; i++) d = max2(d, trd_plane(s, i, p));
    return d;
  }
  if (s->type == OG_SPHERE) {
    double k[S_N];
    sph_comps(s, p, k);
    double d = k[0];
    for (int i = 1; i < S_N; i++) d = max2(d, k[i]);
    return d;
  }
  double k[K_N];
  rad_comps(s, p, k);
  double d = k[0];
  for (int i = 1; i < K_N; i++) d = max2(d, k[i]);
  return d;
}

/* Direction rule for a point on the surface: it is inside only if the
 * direction points strictly inward through every face whose band holds the
 * point.  `vn` values are unnormalised normal components (sign matters). */
static int rad_moving_in(const og_solid* s, const double* p, const double* v, const double k[K_N]) {
  double rho = sqrt(p[0] * p[0] + p[1] * p[1]);
  double rv = rho > 0 ? (p[0] * v[0] + p[1] * v[1]) / rho : 0.0;
  for (int i = 0; i < K_N; i++)
    if (k[i] > -kInf) NOTE_LEN(fabs(k[i]), kHalf);
  if (fabs(k[K_RO]) <= kHalf) {
    double vn = rv - s->Bo * v[2];
    note(vn, 0.0, 1.0);
    if (vn >= 0) return 0;
  }
  if (s->has_inner && fabs(k[K_RI]) <= kHalf) {
    double vn = -rv + s->Bi * v[2];
    note(vn, 0.0, 1.0);
    if (vn >= 0) return 0;
  }
  if (fabs(k[K_Z]) <= kHalf) {
    NOTE_LEN(p[2] * v[2], 0.0);
    if (p[2] * v[2] >= 0) return 0;
  }
  if (s->has_phi) {
    if (fabs(k[K_PA]) <= kHalf) note(v[0] * s->ns[0] + v[1] * s->ns[1], 0.0, 1.0);
    if (fabs(k[K_PA]) <= kHalf && (v[0] * s->ns[0] + v[1] * s->ns[1]) >= 0) return 0;
    if (fabs(k[K_PB]) <= kHalf) note(v[0] * s->ne[0] + v[1] * s->ne[1], 0.0, 1.0);
    if (fabs(k[K_PB]) <= kHalf && (v[0] * s->ne[0] + v[1] * s->ne[1]) >= 0) return 0;
  }
  return 1;
}

/* Classify p (with optional direction v) against the solid. */
int og_solid_inside(const og_solid* s, const double* p, const double* v) {
  double d = og_solid_d(s, p);
  NOTE_LEN(d, d < 0 ? -kHalf : kHalf);
  if (d < -kHalf) return OG_IN;
  if (d > kHalf) return OG_OUT;
  if (!v) return OG_IN;
  if (s->type == OG_BOX) {
    for (int i = 0; i < 3; i++) {
      double si = fabs(p[i]) - s->par[i];
      NOTE_LEN(fabs(si), kHalf);
      if (fabs(si) <= kHalf) NOTE_LEN(p[i] * v[i], 0.0);
      if (fabs(si) <= kHalf && p[i] * v[i] >= 0) return OG_OUT;
    }
    return OG_IN;
  }
  if (s->type == OG_ORB) {
    double b = p[0] * v[0] + p[1] * v[1] + p[2] * v[2];
    NOTE_LEN(b, 0.0);
    return b < 0 ? OG_IN : OG_OUT;
  }
  if (s->type == OG_TRD) {
    for (int i = 0; i < 6; i++) {
      double di = trd_plane(s, i, p);
      NOTE_LEN(fabs(di), kHalf);
      if (fabs(di) <= kHalf) note(trd_dot(s, i, v), 0.0, 1.0);
      if (fabs(di) <= kHalf && trd_dot(s, i, v) >= 0) return OG_OUT;
    }
    return OG_IN;
  }
  if (s->type == OG_SPHERE) {
    double k[S_N];
    sph_comps(s, p, k);
    for (int i = 0; i < S_N; i++) {
      if (!(k[i] > -kInf)) continue;
      NOTE_LEN(fabs(k[i]), kHalf);
      if (fabs(k[i]) > kHalf) continue;
      double dv = sph_comp_dot(s, i, p, v);
      note(dv, 0.0, 1.0);
      if (dv >= 0) return OG_OUT;
    }
    return OG_IN;
  }
  double k[K_N];
  rad_comps(s, p, k);
  return rad_moving_in(s, p, v, k) ? OG_IN : OG_OUT;
}

/* Isotropic safeties: lower bounds on the distance to the solid (from
 * outside) or to its boundary (from inside). */
double og_solid_safety_in(const og_solid* s, const double* p) {
  double d = og_solid_d(s, p);
  return d > 0 ? d : 0.0;
}

double og_solid_safety_out(const og_solid* s, const double* p) {
  double d = og_solid_d(s, p);
  return d < 0 ? -d : 0.0;
}

/* Outward normal of the solid at p (Sec. 3.2: the normal of the boundary
 * surface at the crossing point).  The solid's value is the largest of its
 * face values, so the face that defines the surface at p is the one with the
 * largest value (the first in face order on a tie: box x, y, z; radial
 * outer, inner, z, start phi, end phi), and the normal is that face value's
 * gradient, written out per face below.  Returns the number of faces whose
 * value is within the tolerance of the largest (1 on a face, 2 or more on an
 * edge or corner). */
int og_solid_normal(const og_solid* s, const double* p, double n[3]) {
  double val[6];
  double grad[6][3];
  int nf;
  memset(grad, 0, sizeof(grad));
  if (s->type == OG_BOX) {
    nf = 3;
    for (int i = 0; i < 3; i++) {
      val[i] = fabs(p[i]) - s->par[i];
      grad[i][i] = p[i] < 0 ? -1.0 : 1.0; /* d|p_i|/dp_i */
    }
  } else if (s->type == OG_TRD) {
    /* faces in order +x, -x, +y, -y, +z, -z */
    nf = 6;
    for (int i = 0; i < 6; i++) {
      val[i] = trd_plane(s, i, p);
      for (int c = 0; c < 3; c++) grad[i][c] = s->pn[i][c];
    }
  } else if (s->type == OG_SPHERE) {
    nf = S_N;
    sph_comps(s, p, val);
    double r = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
    double rho = sqrt(p[0] * p[0] + p[1] * p[1]);
    double ex = rho > 0 ? p[0] / rho : 1.0, ey = rho > 0 ? p[1] / rho : 0.0;
    for (int c = 0; c < 3; c++) {
      grad[S_RO][c] = r > 0 ? p[c] / r : (c == 2 ? 1.0 : 0.0);
      grad[S_RI][c] = -grad[S_RO][c];
    }
    grad[S_PA][0] = s->ns[0];
    grad[S_PA][1] = s->ns[1];
    grad[S_PB][0] = s->ne[0];
    grad[S_PB][1] = s->ne[1];
    for (int j = 0; j < 2; j++) {
      double* g = grad[S_T1 + j];
      double c = s->tc[j], B = s->tB[j];
      switch (s->tkind[j]) {
        case T_OUTER: g[0] = c * ex; g[1] = c * ey; g[2] = -c * B; break;
        case T_INNER: g[0] = -c * ex; g[1] = -c * ey; g[2] = c * B; break;
        case T_ZLE: g[2] = 1.0; break;
        case T_ZGE: g[2] = -1.0; break;
        default: break;
      }
    }
  } else if (s->type == OG_ORB) {
    double r = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
    nf = 1;
    val[0] = r - s->par[0];
    if (r > 0) {
      for (int i = 0; i < 3; i++) grad[0][i] = p[i] / r;
    } else {
      grad[0][2] = 1.0;
    }
  } else {
    nf = K_N;
    rad_comps(s, p, val);
    double rho = sqrt(p[0] * p[0] + p[1] * p[1]);
    double ex = rho > 0 ? p[0] / rho : 1.0, ey = rho > 0 ? p[1] / rho : 0.0; /* grad rho */
    /* (rho - (Ao + Bo z)) co */
    grad[K_RO][0] = s->co * ex;
    grad[K_RO][1] = s->co * ey;
    grad[K_RO][2] = -s->co * s->Bo;
    /* ((Ai + Bi z) - rho) ci */
    grad[K_RI][0] = -s->ci * ex;
    grad[K_RI][1] = -s->ci * ey;
    grad[K_RI][2] = s->ci * s->Bi;
    /* |z| - dz */
    grad[K_Z][2] = p[2] < 0 ? -1.0 : 1.0;
    /* p . ns and p . ne */
    grad[K_PA][0] = s->ns[0];
    grad[K_PA][1] = s->ns[1];
    grad[K_PB][0] = s->ne[0];
    grad[K_PB][1] = s->ne[1];
  }
  int best = 0;
  for (int i = 1; i < nf; i++)
    if (val[i] > val[best]) best = i;
  int faces = 0;
  for (int i = 0; i < nf; i++)
    if (val[i] >= val[best] - kTol) faces++;
  for (int i = 0; i < 3; i++) n[i] = grad[best][i];
  return faces;
}

/* Real roots of a t^2 + 2 b t + c, ascending; the numerically stable pair
 * q = -(b + sign(b) sqrt(b^2 - a c)), roots q/a and c/q. */
static int quad_roots(double a, double b, double c, double t[2]) {
  if (a == 0.0) {
    if (b == 0.0) return 0;
    t[0] = -c / (2.0 * b);
    return 1;
  }
  double disc = b * b - a * c;
  note(disc, 0.0, og_scale * og_scale);
  if (disc < 0.0) return 0;
  double sq = sqrt(disc);
  double q = (b >= 0.0) ? -(b + sq) : (sq - b);
  double r1 = q / a;
  double r2 = (q != 0.0) ? c / q : r1;
  if (r1 <= r2) {
    t[0] = r1;
    t[1] = r2;
  } else {
    t[0] = r2;
    t[1] = r1;
  }
  return 2;
}

/* Ray against the radial surface rho = A + B z: coefficients of
 * f(t) = rho(t)^2 - (A + B z(t))^2 = a t^2 + 2 b t + c. */
static void radial_coef(double A, double B, const double* p, const double* v, double* a, double* b,
                        double* c, double* R0, double* Rv) {
  *R0 = A + B * p[2];
  *Rv = B * v[2];
  *a = v[0] * v[0] + v[1] * v[1] - (*Rv) * (*Rv);
  *b = p[0] * v[0] + p[1] * v[1] - (*R0) * (*Rv);
  *c = p[0] * p[0] + p[1] * p[1] - (*R0) * (*R0);
}

/* Smallest root t >= 0 of the radial surface where f'(t) has the requested
 * sign (+1 leaving rho <= R, -1 entering it) on the real sheet R(t) >= 0. */
static double radial_root(double A, double B, const double* p, const double* v, int sign) {
  double a, b, c, R0, Rv, t[2];
  radial_coef(A, B, p, v, &a, &b, &c, &R0, &Rv);
  int n = quad_roots(a, b, c, t);
  double best = kInf;
  for (int i = 0; i < n; i++) {
    double slope = a * t[i] + b;
    NOTE_LEN(slope, 0.0);
    if (sign > 0 ? !(slope > 0) : !(slope < 0)) continue;
    NOTE_LEN(R0 + Rv * t[i], 0.0);
    if (R0 + Rv * t[i] < 0) continue;
    NOTE_LEN(t[i], 0.0);
    if (t[i] < best && t[i] >= 0) best = t[i];
  }
  return best;
}

/* Entering root (f' < 0) on the real sheet, allowing a tiny negative root
 * for a start point inside the surface band (clamped to 0 by the caller). */
static double radial_entry(double A, double B, const double* p, const double* v) {
  double a, b, c, R0, Rv, t[2];
  radial_coef(A, B, p, v, &a, &b, &c, &R0, &Rv);
  int n = quad_roots(a, b, c, t);
  for (int i = 0; i < n; i++) {
    double slope = a * t[i] + b;
    NOTE_LEN(slope, 0.0);
    if (!(slope < 0)) continue;
    NOTE_LEN(R0 + Rv * t[i], 0.0);
    if (R0 + Rv * t[i] < 0) continue;
    return t[i];
  }
  return kInf;
}

/* All components except `skip` hold (within tolerance) at p + t v. */
static int rad_ok_except(const og_solid* s, const double* p, const double* v, double t, int skip) {
  double q[3] = {p[0] + t * v[0], p[1] + t * v[1], p[2] + t * v[2]};
  double k[K_N];
  rad_comps(s, q, k);
  for (int i = 0; i < K_N; i++) {
    if (i == skip) continue;
    if (k[i] > -kInf) NOTE_LEN(k[i], kHalf);
    if (k[i] > kHalf) return 0;
  }
  return 1;
}

static double box_dist_in(const og_solid* s, const double* p, const double* v) {
  for (int i = 0; i < 3; i++) {
    double si = fabs(p[i]) - s->par[i];
    NOTE_LEN(si, -kHalf);
    if (si >= -kHalf) NOTE_LEN(p[i] * v[i], 0.0);
    if (si >= -kHalf && p[i] * v[i] >= 0) return kInf;
  }
  double te = -kInf, tx = kInf;
  for (int i = 0; i < 3; i++) {
    if (v[i] == 0.0) continue;
    double t1 = (-s->par[i] - p[i]) / v[i];
    double t2 = (s->par[i] - p[i]) / v[i];
    double lo = min2(t1, t2), hi = max2(t1, t2);
    te = max2(te, lo);
    tx = min2(tx, hi);
  }
  if (te > -kInf && tx < kInf) NOTE_LEN(te, tx - kHalf);
  if (te >= tx - kHalf) return kInf;
  NOTE_LEN(te, kHalf);
  return te < kHalf ? 0.0 : te;
}

static double box_dist_out(const og_solid* s, const double* p, const double* v) {
  double t = kInf;
  for (int i = 0; i < 3; i++) {
    double sd;
    if (v[i] > 0) sd = s->par[i] - p[i];
    else if (v[i] < 0) sd = s->par[i] + p[i];
    else continue;
    NOTE_LEN(sd, kHalf);
    if (sd <= kHalf) return 0.0;
    t = min2(t, sd / fabs(v[i]));
  }
  return t;
}

static double orb_dist_in(const og_solid* s, const double* p, const double* v) {
  double R = s->par[0];
  double rr = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
  double sd = sqrt(rr) - R;
  double b = p[0] * v[0] + p[1] * v[1] + p[2] * v[2];
  NOTE_LEN(sd, -kHalf);
  if (sd < -kHalf) return 0.0;
  NOTE_LEN(b, 0.0);
  if (b >= 0) return kInf;
  double c = rr - R * R;
  double disc = b * b - c;
  note(disc, 0.0, og_scale * og_scale);
  if (disc <= 0) return kInf;
  double sq = sqrt(disc);
  double te = c / (sq - b);
  double tx = sq - b;
  NOTE_LEN(te, tx - kHalf);
  if (te >= tx - kHalf) return kInf;
  NOTE_LEN(te, kHalf);
  return te < kHalf ? 0.0 : te;
}

static double orb_dist_out(const og_solid* s, const double* p, const double* v) {
  double R = s->par[0];
  double rr = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
  double sd = sqrt(rr) - R;
  double b = p[0] * v[0] + p[1] * v[1] + p[2] * v[2];
  NOTE_LEN(sd, -kHalf);
  if (sd >= -kHalf) NOTE_LEN(b, 0.0);
  if (sd >= -kHalf && b >= 0) return 0.0;
  double c = rr - R * R;
  double disc = b * b - c;
  if (disc < 0) disc = 0;
  double sq = sqrt(disc);
  double t = (b > 0) ? -c / (b + sq) : sq - b;
  return t > 0 ? t : 0.0;
}

/* Distance along v to entering a tube or cone section, surface by surface:
 * for each face crossed inward, keep the crossing if every other component
 * holds there.  A start point on the band moving in gives 0. */
static double rad_dist_in(const og_solid* s, const double* p, const double* v) {
  double k[K_N];
  rad_comps(s, p, k);
  double d = k[0];
  for (int i = 1; i < K_N; i++) d = max2(d, k[i]);
  NOTE_LEN(d, -kHalf);
  if (d < -kHalf) return 0.0;
  double rho = sqrt(p[0] * p[0] + p[1] * p[1]);
  double rv = rho > 0 ? (p[0] * v[0] + p[1] * v[1]) / rho : 0.0;
  double best = kInf;
  for (int i = 0; i < K_N; i++)
    if (k[i] > -kInf) NOTE_LEN(k[i], -kHalf);
  /* z planes */
  if (k[K_Z] >= -kHalf) {
    NOTE_LEN(p[2] * v[2], 0.0);
    if (p[2] * v[2] >= 0) return kInf;
    double t = k[K_Z] / fabs(v[2]);
    if (t < 0) t = 0;
    if (rad_ok_except(s, p, v, t, K_Z)) best = min2(best, t);
  }
  /* outer radial surface (convex region) */
  if (k[K_RO] >= -kHalf) {
    double vn = rv - s->Bo * v[2];
    note(vn, 0.0, 1.0);
    if (vn >= 0) return kInf;
    double t = radial_entry(s->Ao, s->Bo, p, v);
    if (t == kInf) return kInf;
    if (t < 0) t = 0;
    if (rad_ok_except(s, p, v, t, K_RO)) best = min2(best, t);
  }
  /* inner radial surface: entering the section from its bore */
  if (s->has_inner) {
    double t = -1.0;
    NOTE_LEN(fabs(k[K_RI]), kHalf);
    if (fabs(k[K_RI]) <= kHalf) {
      double vn = -rv + s->Bi * v[2];
      note(vn, 0.0, 1.0);
      if (vn < 0) t = 0.0;
      else if (vn > 0) t = radial_root(s->Ai, s->Bi, p, v, +1);
    } else {
      t = radial_root(s->Ai, s->Bi, p, v, +1);
    }
    if (t >= 0 && t < kInf && rad_ok_except(s, p, v, t, K_RI)) best = min2(best, t);
  }
  /* phi planes (wedge no wider than pi: convex) */
  if (s->has_phi) {
    for (int q = 0; q < 2; q++) {
      const double* n = q == 0 ? s->ns : s->ne;
      double dp = q == 0 ? k[K_PA] : k[K_PB];
      if (dp >= -kHalf) {
        double dv = v[0] * n[0] + v[1] * n[1];
        note(dv, 0.0, 1.0);
        if (dv >= 0) return kInf;
        double t = dp / (-dv);
        if (t < 0) t = 0;
        if (rad_ok_except(s, p, v, t, q == 0 ? K_PA : K_PB)) best = min2(best, t);
      }
    }
  }
  if (best < kInf) NOTE_LEN(best, kHalf);
  return best < kHalf ? 0.0 : best;
}

/* Distance along v to leaving a tube or cone section: the first exit over
 * its components; 0 when on a face band and not moving strictly inward. */
static double rad_dist_out(const og_solid* s, const double* p, const double* v) {
  double k[K_N];
  rad_comps(s, p, k);
  double rho = sqrt(p[0] * p[0] + p[1] * p[1]);
  double rv = rho > 0 ? (p[0] * v[0] + p[1] * v[1]) / rho : 0.0;
  double t = kInf;
  if (v[2] != 0) {
    double sd = v[2] > 0 ? s->dz - p[2] : s->dz + p[2];
    NOTE_LEN(sd, kHalf);
    if (sd <= kHalf) return 0.0;
    t = min2(t, sd / fabs(v[2]));
  }
  NOTE_LEN(k[K_RO], -kHalf);
  if (k[K_RO] >= -kHalf) note(rv - s->Bo * v[2], 0.0, 1.0);
  if (k[K_RO] >= -kHalf && rv - s->Bo * v[2] >= 0) return 0.0;
  t = min2(t, radial_root(s->Ao, s->Bo, p, v, +1));
  if (s->has_inner) {
    NOTE_LEN(k[K_RI], -kHalf);
    if (k[K_RI] >= -kHalf) note(-rv + s->Bi * v[2], 0.0, 1.0);
    if (k[K_RI] >= -kHalf && -rv + s->Bi * v[2] >= 0) return 0.0;
    t = min2(t, radial_root(s->Ai, s->Bi, p, v, -1));
  }
  if (s->has_phi) {
    for (int q = 0; q < 2; q++) {
      const double* n = q == 0 ? s->ns : s->ne;
      double dp = q == 0 ? k[K_PA] : k[K_PB];
      double dv = v[0] * n[0] + v[1] * n[1];
      NOTE_LEN(dp, -kHalf);
      note(dv, 0.0, 1.0);
      if (dp >= -kHalf && dv >= 0) return 0.0;
      if (dv > 0) {
        double tp = -dp / dv;
        if (tp < 0) tp = 0;
        t = min2(t, tp);
      }
    }
  }
  return t;
}

/* Trapezoid, a convex solid of six planes: entering distance as the latest
 * plane entry before the earliest plane exit, with the box's tolerance rules
 * (a face whose band holds p, or beyond it, that the ray does not cross
 * inward can never be crossed: no entry; a start point on the band moving in
 * gives 0). */
static double trd_dist_in(const og_solid* s, const double* p, const double* v) {
  double dv[6], dp[6];
  for (int i = 0; i < 6; i++) {
    dp[i] = trd_plane(s, i, p);
    dv[i] = trd_dot(s, i, v);
    NOTE_LEN(dp[i], -kHalf);
    if (dp[i] >= -kHalf) note(dv[i], 0.0, 1.0);
    if (dp[i] >= -kHalf && dv[i] >= 0) return kInf;
  }
  double te = -kInf, tx = kInf;
  for (int i = 0; i < 6; i++) {
    if (dv[i] == 0.0) continue;
    double t = -dp[i] / dv[i];
    if (dv[i] < 0) te = max2(te, t);
    else tx = min2(tx, t);
  }
  if (te > -kInf && tx < kInf) NOTE_LEN(te, tx - kHalf);
  if (te >= tx - kHalf) return kInf;
  NOTE_LEN(te, kHalf);
  return te < kHalf ? 0.0 : te;
}

/* All sphere components except `skip` hold (within tolerance) at p + t v. */
static int sph_ok_except(const og_solid* s, const double* p, const double* v, double t, int skip) {
  double q[3] = {p[0] + t * v[0], p[1] + t * v[1], p[2] + t * v[2]};
  double k[S_N];
  sph_comps(s, q, k);
  for (int i = 0; i < S_N; i++) {
    if (i == skip) continue;
    if (k[i] > -kInf) NOTE_LEN(k[i], kHalf);
    if (k[i] > kHalf) return 0;
  }
  return 1;
}

/* Sphere section entry, surface by surface (as for tube and cone sections): a
 * crossing through one face counts if every other component holds there.
 * The regions r <= rmax, a phi wedge, the inside of a cone and a half-space
 * are convex, so a ray that does not cross one of those faces inward from
 * its band or beyond never enters; r >= rmin and the outside of a cone are
 * not. */
static double sph_dist_in(const og_solid* s, const double* p, const double* v) {
  double k[S_N];
  sph_comps(s, p, k);
  double d = k[0];
  for (int i = 1; i < S_N; i++) d = max2(d, k[i]);
  NOTE_LEN(d, -kHalf);
  if (d < -kHalf) return 0.0;
  double rr = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
  double b = p[0] * v[0] + p[1] * v[1] + p[2] * v[2];
  double best = kInf;
  for (int i = 0; i < S_N; i++)
    if (k[i] > -kInf) NOTE_LEN(k[i], -kHalf);
  /* outer sphere: the ball's entry */
  if (k[S_RO] >= -kHalf) {
    NOTE_LEN(b, 0.0);
    if (b >= 0) return kInf;
    double c = rr - s->srmax * s->srmax;
    double disc = b * b - c;
    note(disc, 0.0, og_scale * og_scale);
    if (disc <= 0) return kInf;
    double sq = sqrt(disc);
    double t = c / (sq - b);
    if (t < 0) t = 0;
    if (sph_ok_except(s, p, v, t, S_RO)) best = min2(best, t);
  }
  /* inner sphere: leaving the inner ball */
  if (s->has_inner) {
    double t = -1.0;
    double c = rr - s->srmin * s->srmin;
    double disc = b * b - c;
    NOTE_LEN(fabs(k[S_RI]), kHalf);
    if (fabs(k[S_RI]) <= kHalf) {
      NOTE_LEN(b, 0.0);
      if (b > 0) t = 0.0;
      else if (b < 0 && disc > 0) t = sqrt(disc) - b;
    } else if (disc > 0) {
      double sq = sqrt(disc);
      t = (b > 0) ? -c / (b + sq) : sq - b;
    }
    if (t >= 0 && t < kInf && sph_ok_except(s, p, v, t, S_RI)) best = min2(best, t);
  }
  /* phi planes (wedge no wider than pi: convex) */
  if (s->has_phi) {
    for (int q = 0; q < 2; q++) {
      const double* n = q == 0 ? s->ns : s->ne;
      double dp = q == 0 ? k[S_PA] : k[S_PB];
      if (dp >= -kHalf) {
        double dv = v[0] * n[0] + v[1] * n[1];
        note(dv, 0.0, 1.0);
        if (dv >= 0) return kInf;
        double t = dp / (-dv);
        if (t < 0) t = 0;
        if (sph_ok_except(s, p, v, t, q == 0 ? S_PA : S_PB)) best = min2(best, t);
      }
    }
  }
  /* theta bounds */
  for (int j = 0; j < 2; j++) {
    const int i = S_T1 + j;
    const int kind = s->tkind[j];
    if (kind == T_NONE) continue;
    if (kind == T_OUTER) {
      if (k[i] >= -kHalf) {
        double vn = sph_comp_dot(s, i, p, v);
        note(vn, 0.0, 1.0);
        if (vn >= 0) return kInf;
        double t = radial_entry(0.0, s->tB[j], p, v);
        if (t == kInf) return kInf;
        if (t < 0) t = 0;
        if (sph_ok_except(s, p, v, t, i)) best = min2(best, t);
      }
    } else if (kind == T_INNER) {
      double t = -1.0;
      NOTE_LEN(fabs(k[i]), kHalf);
      if (fabs(k[i]) <= kHalf) {
        double vn = sph_comp_dot(s, i, p, v);
        note(vn, 0.0, 1.0);
        if (vn < 0) t = 0.0;
        else if (vn > 0) t = radial_root(0.0, s->tB[j], p, v, +1);
      } else {
        t = radial_root(0.0, s->tB[j], p, v, +1);
      }
      if (t >= 0 && t < kInf && sph_ok_except(s, p, v, t, i)) best = min2(best, t);
    } else {
      /* half-space z <= 0 (T_ZLE) or z >= 0 (T_ZGE), component k = +-z */
      if (k[i] >= -kHalf) {
        double vn = kind == T_ZLE ? v[2] : -v[2];
        NOTE_LEN(vn, 0.0);
        if (vn >= 0) return kInf;
        double t = k[i] / (-vn);
        if (t < 0) t = 0;
        if (sph_ok_except(s, p, v, t, i)) best = min2(best, t);
      }
    }
  }
  if (best < kInf) NOTE_LEN(best, kHalf);
  return best < kHalf ? 0.0 : best;
}

/* Sphere section exit: the first outward crossing over its components; 0 on
 * a face band when not moving strictly inward. */
static double sph_dist_out(const og_solid* s, const double* p, const double* v) {
  double k[S_N];
  sph_comps(s, p, k);
  double rr = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
  double b = p[0] * v[0] + p[1] * v[1] + p[2] * v[2];
  double t = kInf;
  /* outer sphere */
  NOTE_LEN(k[S_RO], -kHalf);
  if (k[S_RO] >= -kHalf) NOTE_LEN(b, 0.0);
  if (k[S_RO] >= -kHalf && b >= 0) return 0.0;
  {
    double c = rr - s->srmax * s->srmax;
    double disc = b * b - c;
    if (disc < 0) disc = 0;
    double sq = sqrt(disc);
    double to = (b > 0) ? -c / (b + sq) : sq - b;
    t = min2(t, to > 0 ? to : 0.0);
  }
  /* inner sphere: entering the inner ball */
  if (s->has_inner) {
    NOTE_LEN(k[S_RI], -kHalf);
    if (k[S_RI] >= -kHalf) NOTE_LEN(b, 0.0);
    if (k[S_RI] >= -kHalf && b <= 0) return 0.0;
    if (b < 0) {
      double c = rr - s->srmin * s->srmin;
      double disc = b * b - c;
      note(disc, 0.0, og_scale * og_scale);
      if (disc > 0) {
        double ti = c / (sqrt(disc) - b);
        t = min2(t, ti > 0 ? ti : 0.0);
      }
    }
  }
  if (s->has_phi) {
    for (int q = 0; q < 2; q++) {
      const double* n = q == 0 ? s->ns : s->ne;
      double dp = q == 0 ? k[S_PA] : k[S_PB];
      double dv = v[0] * n[0] + v[1] * n[1];
      NOTE_LEN(dp, -kHalf);
      note(dv, 0.0, 1.0);
      if (dp >= -kHalf && dv >= 0) return 0.0;
      if (dv > 0) {
        double tp = -dp / dv;
        if (tp < 0) tp = 0;
        t = min2(t, tp);
      }
    }
  }
  for (int j = 0; j < 2; j++) {
    const int i = S_T1 + j;
    const int kind = s->tkind[j];
    if (kind == T_NONE) continue;
    double vn = sph_comp_dot(s, i, p, v);
    NOTE_LEN(k[i], -kHalf);
    note(vn, 0.0, 1.0);
    if (k[i] >= -kHalf && vn >= 0) return 0.0;
    if (kind == T_OUTER) {
      t = min2(t, radial_root(0.0, s->tB[j], p, v, +1));
    } else if (kind == T_INNER) {
      t = min2(t, radial_root(0.0, s->tB[j], p, v, -1));
    } else if (vn > 0) {
      double sd = -k[i];
      NOTE_LEN(sd, kHalf);
      if (sd <= kHalf) return 0.0;
      t = min2(t, sd / vn);
    }
  }
  return t;
}

/* Leaving distance: the earliest plane exit; 0 on a face band moving out. */
static double trd_dist_out(const og_solid* s, const double* p, const double* v) {
  double t = kInf;
  for (int i = 0; i < 6; i++) {
    double dv = trd_dot(s, i, v);
    if (!(dv > 0)) continue;
    double sd = -trd_plane(s, i, p);
    NOTE_LEN(sd, kHalf);
    if (sd <= kHalf) return 0.0;
    t = min2(t, sd / dv);
  }
  return t;
}

double og_solid_dist_in(const og_solid* s, const double* p, const double* v) {
  switch (s->type) {
    case OG_BOX: return box_dist_in(s, p, v);
    case OG_ORB: return orb_dist_in(s, p, v);
    case OG_TRD: return trd_dist_in(s, p, v);
    case OG_SPHERE: return sph_dist_in(s, p, v);
    default: return rad_dist_in(s, p, v);
  }
}

double og_solid_dist_out(const og_solid* s, const double* p, const double* v) {
  switch (s->type) {
    case OG_BOX: return box_dist_out(s, p, v);
    case OG_ORB: return orb_dist_out(s, p, v);
    case OG_TRD: return trd_dist_out(s, p, v);
    case OG_SPHERE: return sph_dist_out(s, p, v);
    default: return rad_dist_out(s, p, v);
  }
}

/* ------------------------------------------------------------------------ */
/* Geometry: logical volumes, placements and touchables.                     */
/* ------------------------------------------------------------------------ */

typedef struct {
  int n_solids;
  og_solid* solids;
  int n_mats;
  double* density;
  double* tab; /* [n_mats][3][OG_NNODE] attenuation, 1/mm */
  double lnE0, dlnE;
  int n_lv;
  int *lv_solid, *lv_mat, *lv_dau_off, *lv_dau_cnt;
  int n_pv;
  int* pv_lv;
  double *pv_rot, *pv_trans;
  int world_lv;
  int n_t;
  int *t_parent, *t_pv, *t_slot, *t_lv, *t_child_base, *t_depth;
  /* mode: 0 = physics tables, 1 = paper mode mu = rho * mu_mass (single process) */
  int paper_mode;
  double paper_mu_mass; /* cm2/g */
  /* voxel mode (faster CPU search, same answers): per-LV cell grids */
  struct og_vgrid* vgrid; /* [n_lv] or NULL */
  int use_voxels;
} og_geom;

static void* xcalloc(size_t n, size_t sz) {
  void* p = calloc(n ? n : 1, sz);
  return p;
}

static void to_local(const double* R, const double* t, const double* pm, double* pl) {
  double d0 = pm[0] - t[0], d1 = pm[1] - t[1], d2 = pm[2] - t[2];
  pl[0] = R[0] * d0 + R[3] * d1 + R[6] * d2;
  pl[1] = R[1] * d0 + R[4] * d1 + R[7] * d2;
  pl[2] = R[2] * d0 + R[5] * d1 + R[8] * d2;
}

static void dir_to_local(const double* R, const double* vm, double* vl) {
  vl[0] = R[0] * vm[0] + R[3] * vm[1] + R[6] * vm[2];
  vl[1] = R[1] * vm[0] + R[4] * vm[1] + R[7] * vm[2];
  vl[2] = R[2] * vm[0] + R[5] * vm[1] + R[8] * vm[2];
}

/* mu per process of material m at energy E (1/mm), tabulated on 257
 * log-spaced nodes and interpolated linearly in ln E; pair is zero below
 * its threshold 2 m_e c^2. */
static void build_tables(og_geom* g, const double* density, const int* el_off, const int* el_Z,
                         const double* el_A, const double* el_w) {
  g->lnE0 = log(1e-3);
  g->dlnE = log(1e5) / 256.0;
  g->tab = (double*)xcalloc((size_t)g->n_mats * 3 * OG_NNODE, sizeof(double));
  for (int m = 0; m < g->n_mats; m++) {
    for (int i = 0; i < OG_NNODE; i++) {
      long double E = expl((long double)g->lnE0 + (long double)i * (long double)g->dlnE);
      long double mu[3] = {0, 0, 0};
      for (int e = el_off[m]; e < el_off[m + 1]; e++) {
        double sg[3];
        og_sigma_atom(el_Z[e], (double)E, sg);
        long double n_atoms = (long double)density[m] * kNaL * (long double)el_w[e] / (long double)el_A[e];
        for (int p = 0; p < 3; p++) mu[p] += n_atoms * (long double)sg[p];
      }
      for (int p = 0; p < 3; p++) g->tab[((size_t)m * 3 + p) * OG_NNODE + i] = (double)(mu[p] * 0.1L);
    }
  }
}

static void mu_lookup(const og_geom* g, int mat, double E, double mu[3]) {
  if (g->paper_mode) {
    mu[0] = 0.0;
    mu[1] = g->density[mat] * g->paper_mu_mass * 0.1;
    mu[2] = 0.0;
    return;
  }
  double x = (log(E) - g->lnE0) / g->dlnE;
  int i;
  if (x < 0) i = 0;
  else if (x >= 255.0) i = 255;
  else i = (int)x;
  double w = x - (double)i;
  if (w < 0) w = 0;
  if (w > 1) w = 1;
  const double* t = g->tab + (size_t)mat * 3 * OG_NNODE;
  for (int p = 0; p < 3; p++) mu[p] = (1.0 - w) * t[p * OG_NNODE + i] + w * t[p * OG_NNODE + i + 1];
  if (E < 2.0 * kMe) mu[2] = 0.0;
}

void og_destroy(og_geom* g);
static void og_free_voxels(og_geom* g);

/* Build the oracle's geometry from the flat description.  Touchables are
 * numbered breadth first from the world (0): the children of touchable T
 * are child_base[T] + slot, slot being the placement's index in its mother. */
og_geom* og_create(int n_solids, const int* solid_type, const double* solid_par, int n_mats,
                   const double* density, const int* el_off, const int* el_Z, const double* el_A,
                   const double* el_w, int n_lv, const int* lv_solid, const int* lv_mat,
                   const int* lv_dau_off, const int* lv_dau_cnt, int n_pv, const int* pv_lv,
                   const double* pv_rot, const double* pv_trans, int world_lv) {
  og_geom* g = (og_geom*)xcalloc(1, sizeof(og_geom));
  g->n_solids = n_solids;
  g->solids = (og_solid*)xcalloc(n_solids, sizeof(og_solid));
  for (int i = 0; i < n_solids; i++) {
    if (solid_init(&g->solids[i], solid_type[i], solid_par + 8 * i) != 0) {
      og_destroy(g);
      return NULL;
    }
  }
  g->n_mats = n_mats;
  g->density = (double*)xcalloc(n_mats, sizeof(double));
  memcpy(g->density, density, n_mats * sizeof(double));
  build_tables(g, density, el_off, el_Z, el_A, el_w);
  g->n_lv = n_lv;
  g->lv_solid = (int*)xcalloc(n_lv, sizeof(int));
  g->lv_mat = (int*)xcalloc(n_lv, sizeof(int));
  g->lv_dau_off = (int*)xcalloc(n_lv, sizeof(int));
  g->lv_dau_cnt = (int*)xcalloc(n_lv, sizeof(int));
  memcpy(g->lv_solid, lv_solid, n_lv * sizeof(int));
  memcpy(g->lv_mat, lv_mat, n_lv * sizeof(int));
  memcpy(g->lv_dau_off, lv_dau_off, n_lv * sizeof(int));
  memcpy(g->lv_dau_cnt, lv_dau_cnt, n_lv * sizeof(int));
  g->n_pv = n_pv;
  g->pv_lv = (int*)xcalloc(n_pv, sizeof(int));
  g->pv_rot = (double*)xcalloc((size_t)n_pv * 9, sizeof(double));
  g->pv_trans = (double*)xcalloc((size_t)n_pv * 3, sizeof(double));
  memcpy(g->pv_lv, pv_lv, n_pv * sizeof(int));
  memcpy(g->pv_rot, pv_rot, (size_t)n_pv * 9 * sizeof(double));
  memcpy(g->pv_trans, pv_trans, (size_t)n_pv * 3 * sizeof(double));
  g->world_lv = world_lv;
  for (int l = 0; l < n_lv; l++) {
    if (lv_solid[l] < 0 || lv_solid[l] >= n_solids || lv_mat[l] < 0 || lv_mat[l] >= n_mats ||
        lv_dau_off[l] < 0 || lv_dau_cnt[l] < 0 || lv_dau_off[l] + lv_dau_cnt[l] > n_pv) {
      og_destroy(g);
      return NULL;
    }
  }
  /* count touchables */
  long long cap = 1;
  {
    long long* cnt = (long long*)xcalloc(n_lv, sizeof(long long));
    /* LVs can be nested arbitrarily; count by repeated relaxation (DAG). */
    for (int it = 0; it < 64; it++) {
      int changed = 0;
      for (int l = 0; l < n_lv; l++) {
        long long c = 1;
        for (int k = 0; k < lv_dau_cnt[l]; k++) c += cnt[pv_lv[lv_dau_off[l] + k]];
        if (c != cnt[l]) {
          cnt[l] = c;
          changed = 1;
        }
      }
      if (!changed) break;
    }
    cap = cnt[world_lv];
    free(cnt);
  }
  if (cap > (1LL << 30)) {
    og_destroy(g);
    return NULL;
  }
  int n = (int)cap;
  g->t_parent = (int*)xcalloc(n, sizeof(int));
  g->t_pv = (int*)xcalloc(n, sizeof(int));
  g->t_slot = (int*)xcalloc(n, sizeof(int));
  g->t_lv = (int*)xcalloc(n, sizeof(int));
  g->t_child_base = (int*)xcalloc(n, sizeof(int));
  g->t_depth = (int*)xcalloc(n, sizeof(int));
  int cnt = 1;
  g->t_parent[0] = -1;
  g->t_pv[0] = -1;
  g->t_slot[0] = -1;
  g->t_lv[0] = world_lv;
  g->t_depth[0] = 0;
  for (int i = 0; i < cnt; i++) {
    int l = g->t_lv[i];
    g->t_child_base[i] = cnt;
    for (int k = 0; k < lv_dau_cnt[l]; k++) {
      int pv = lv_dau_off[l] + k;
      g->t_parent[cnt] = i;
      g->t_pv[cnt] = pv;
      g->t_slot[cnt] = k;
      g->t_lv[cnt] = pv_lv[pv];
      g->t_depth[cnt] = g->t_depth[i] + 1;
      cnt++;
    }
  }
  g->n_t = cnt;
  return g;
}

void og_destroy(og_geom* g) {
  if (!g) return;
  free(g->solids);
  free(g->density);
  free(g->tab);
  free(g->lv_solid);
  free(g->lv_mat);
  free(g->lv_dau_off);
  free(g->lv_dau_cnt);
  free(g->pv_lv);
  free(g->pv_rot);
  free(g->pv_trans);
  free(g->t_parent);
  free(g->t_pv);
  free(g->t_slot);
  free(g->t_lv);
  free(g->t_child_base);
  free(g->t_depth);
  og_free_voxels(g);
  free(g);
}

int og_n_touchables(const og_geom* g) { return g->n_t; }

void og_touchables(const og_geom* g, int* parent, int* pv, int* lv, int* depth) {
  for (int i = 0; i < g->n_t; i++) {
    if (parent) parent[i] = g->t_parent[i];
    if (pv) pv[i] = g->t_pv[i];
    if (lv) lv[i] = g->t_lv[i];
    if (depth) depth[i] = g->t_depth[i];
  }
}

void og_set_paper_mode(og_geom* g, int on, double mu_mass_cm2_per_g) {
  g->paper_mode = on;
  g->paper_mu_mass = mu_mass_cm2_per_g;
}

void og_mu(const og_geom* g, int mat, int n, const double* E, double* out /*[n][3]*/) {
  for (int i = 0; i < n; i++) mu_lookup(g, mat, E[i], out + 3 * i);
}

void og_table(const og_geom* g, double* out /*[n_mats][3][257]*/, double* lnE0, double* dlnE) {
  memcpy(out, g->tab, (size_t)g->n_mats * 3 * OG_NNODE * sizeof(double));
  *lnE0 = g->lnE0;
  *dlnE = g->dlnE;
}

/* Point and direction in the frame of touchable T, applying the inverse
 * placements level by level from the world down. */
static void frame_of(const og_geom* g, int T, const double* pg, const double* vg, double* pl, double* vl) {
  int chain[64];
  int n = 0;
  for (int u = T; u > 0; u = g->t_parent[u]) chain[n++] = u;
  double p[3] = {pg[0], pg[1], pg[2]}, v[3] = {0, 0, 0};
  if (vg) {
    v[0] = vg[0];
    v[1] = vg[1];
    v[2] = vg[2];
  }
  for (int i = n - 1; i >= 0; i--) {
    int pv = g->t_pv[chain[i]];
    double q[3], w[3];
    to_local(g->pv_rot + 9 * pv, g->pv_trans + 3 * pv, p, q);
    memcpy(p, q, sizeof(q));
    if (vg) {
      dir_to_local(g->pv_rot + 9 * pv, v, w);
      memcpy(v, w, sizeof(w));
    }
  }
  memcpy(pl, p, sizeof(p));
  if (vl) memcpy(vl, v, sizeof(v));
}

static const og_solid* lv_solid_of(const og_geom* g, int lv) { return &g->solids[g->lv_solid[lv]]; }

/* ------------------------------------------------------------------------ */
/* Voxel mode: the oracle's own faster search, for CPU timing.               */
/*                                                                           */
/* A uniform grid over each mother's bounding box lists, per cell and in     */
/* ascending slot order, the daughters whose bounding box grown by           */
/* kVoxMargin meets the cell (tubs and cons placed along the mother's z axis */
/* also need the cell to meet their radial range, orbs their sphere).  Any   */
/* daughter that holds a point, or whose surface band the ray reaches while  */
/* still inside the cells visited so far, is listed in those cells, so       */
/* locate and ComputeStep give exactly the brute-force answers.  The GPU     */
/* library's voxels are built independently and differently.                 */
/* ------------------------------------------------------------------------ */

static const double kVoxMargin = 1e-6;

typedef struct og_vgrid {
  int n[3];
  double lo[3], w[3];
  int* off; /* [cells + 1], NULL: no grid (brute force) */
  int* dau;
} og_vgrid;

/* Bounding box of a solid in its own frame.  A phi segment of a tubs or
 * cons is bounded by its corner points and by the outer radius at the axis
 * directions the segment spans. */
static void solid_box(const og_solid* s, double lo[3], double hi[3]) {
  const double* p = s->par;
  if (s->type == OG_TRD) {
    const double hx = max2(p[0], p[1]), hy = max2(p[2], p[3]);
    lo[0] = -hx;
    hi[0] = hx;
    lo[1] = -hy;
    hi[1] = hy;
    lo[2] = -p[4];
    hi[2] = p[4];
    return;
  }
  if (s->type == OG_SPHERE) {
    for (int i = 0; i < 3; i++) {
      lo[i] = -p[1];
      hi[i] = p[1];
    }
    return;
  }
  if (s->type == OG_BOX || s->type == OG_ORB) {
    for (int i = 0; i < 3; i++) {
      double h = s->type == OG_BOX ? p[i] : p[0];
      lo[i] = -h;
      hi[i] = h;
    }
    return;
  }
  double rin = s->type == OG_TUBS ? p[0] : min2(p[0], p[2]);
  double rout = s->type == OG_TUBS ? p[1] : max2(p[1], p[3]);
  double dz = s->type == OG_TUBS ? p[2] : p[4];
  double sphi = s->type == OG_TUBS ? p[3] : p[5];
  double dphi = s->type == OG_TUBS ? p[4] : p[6];
  lo[2] = -dz;
  hi[2] = dz;
  if (!s->has_phi) {
    lo[0] = lo[1] = -rout;
    hi[0] = hi[1] = rout;
    return;
  }
  lo[0] = lo[1] = kInf;
  hi[0] = hi[1] = -kInf;
  const double ang[2] = {sphi, sphi + dphi};
  for (int a = 0; a < 2; a++)
    for (int r = 0; r < 2; r++) {
      double rr = r ? rout : rin, x = rr * cos(ang[a]), y = rr * sin(ang[a]);
      lo[0] = min2(lo[0], x);
      hi[0] = max2(hi[0], x);
      lo[1] = min2(lo[1], y);
      hi[1] = max2(hi[1], y);
    }
  for (int k = -8; k <= 8; k++) {
    double a = k * (M_PI / 2);
    if (a < sphi || a > sphi + dphi) continue;
    int q = ((k % 4) + 4) % 4; /* +x, +y, -x, -y */
    if (q == 0) hi[0] = rout;
    if (q == 1) hi[1] = rout;
    if (q == 2) lo[0] = -rout;
    if (q == 3) lo[1] = -rout;
  }
}

/* Does daughter pv (of solid s) possibly meet the cell [c0, c1] (mother frame)? */
static int dau_meets_cell(const og_geom* g, int pv, const double c0[3], const double c1[3]) {
  const og_solid* s = lv_solid_of(g, g->pv_lv[pv]);
  const double* R = g->pv_rot + 9 * pv;
  const double* t = g->pv_trans + 3 * pv;
  const double m = kVoxMargin;
  if (s->type == OG_ORB) {
    double d2 = 0;
    for (int i = 0; i < 3; i++) {
      double d = max2(max2(c0[i] - t[i], t[i] - c1[i]), 0.0);
      d2 += d * d;
    }
    return sqrt(d2) <= s->par[0] + m;
  }
  if ((s->type == OG_TUBS || s->type == OG_CONS) && fabs(R[8]) == 1.0) {
    /* axis parallel to the mother's z: compare the cell's xy distances
     * from the axis with the solid's radial range */
    double dx = max2(max2(c0[0] - t[0], t[0] - c1[0]), 0.0);
    double dy = max2(max2(c0[1] - t[1], t[1] - c1[1]), 0.0);
    double dmin = sqrt(dx * dx + dy * dy);
    double fx = max2(fabs(c0[0] - t[0]), fabs(c1[0] - t[0]));
    double fy = max2(fabs(c0[1] - t[1]), fabs(c1[1] - t[1]));
    double dmax = sqrt(fx * fx + fy * fy);
    double rin = s->type == OG_TUBS ? s->par[0] : min2(s->par[0], s->par[2]);
    double rout = s->type == OG_TUBS ? s->par[1] : max2(s->par[1], s->par[3]);
    if (dmin > rout + m || dmax < rin - m) return 0;
  }
  return 1;
}

static void og_free_voxels(og_geom* g) {
  if (!g->vgrid) return;
  for (int l = 0; l < g->n_lv; l++) {
    free(g->vgrid[l].off);
    free(g->vgrid[l].dau);
  }
  free(g->vgrid);
  g->vgrid = NULL;
}

/* Build the grid of one mother LV with nd >= 4 daughters: about 64 cells per
 * daughter (at most 2^20), cubic cells where the extents allow. */
static int build_grid(og_geom* g, int lv, og_vgrid* G) {
  int nd = g->lv_dau_cnt[lv];
  double mlo[3], mhi[3];
  solid_box(lv_solid_of(g, lv), mlo, mhi);
  double vol = (mhi[0] - mlo[0]) * (mhi[1] - mlo[1]) * (mhi[2] - mlo[2]);
  double target = min2(64.0 * nd, 1048576.0);
  double edge = cbrt(vol / target);
  long cells = 1;
  for (int i = 0; i < 3; i++) {
    int n = (int)ceil((mhi[i] - mlo[i]) / edge);
    n = n < 1 ? 1 : (n > 1024 ? 1024 : n);
    G->n[i] = n;
    G->lo[i] = mlo[i];
    G->w[i] = (mhi[i] - mlo[i]) / n;
    cells *= n;
  }
  if (cells > 4 * 1048576L) return -1;
  int* cnt = (int*)xcalloc((size_t)cells + 1, sizeof(int));
  /* two passes over the daughters: count, then fill in slot order */
  long total = 0;
  for (int pass = 0; pass < 2; pass++) {
    for (int k = 0; k < nd; k++) {
      int pv = g->lv_dau_off[lv] + k;
      double blo[3], bhi[3], cl[3], hd[3], lo[3], hi[3];
      solid_box(lv_solid_of(g, g->pv_lv[pv]), blo, bhi);
      for (int i = 0; i < 3; i++) {
        cl[i] = 0.5 * (blo[i] + bhi[i]);
        hd[i] = 0.5 * (bhi[i] - blo[i]);
      }
      const double* R = g->pv_rot + 9 * pv;
      const double* t = g->pv_trans + 3 * pv;
      int i0[3], i1[3];
      for (int i = 0; i < 3; i++) {
        /* mother-frame box of the placed local box: centre R cl + t, half |R| hd */
        double cm = R[3 * i] * cl[0] + R[3 * i + 1] * cl[1] + R[3 * i + 2] * cl[2] + t[i];
        double e = fabs(R[3 * i]) * hd[0] + fabs(R[3 * i + 1]) * hd[1] + fabs(R[3 * i + 2]) * hd[2];
        lo[i] = cm - e - kVoxMargin - 1e-9 * fabs(cm);
        hi[i] = cm + e + kVoxMargin + 1e-9 * fabs(cm);
        double a = floor((lo[i] - G->lo[i]) / G->w[i]), b = floor((hi[i] - G->lo[i]) / G->w[i]);
        i0[i] = a < 0 ? 0 : (a > G->n[i] - 1 ? G->n[i] - 1 : (int)a);
        i1[i] = b < 0 ? 0 : (b > G->n[i] - 1 ? G->n[i] - 1 : (int)b);
      }
      for (int ix = i0[0]; ix <= i1[0]; ix++)
        for (int iy = i0[1]; iy <= i1[1]; iy++)
          for (int iz = i0[2]; iz <= i1[2]; iz++) {
            double c0[3] = {G->lo[0] + ix * G->w[0], G->lo[1] + iy * G->w[1], G->lo[2] + iz * G->w[2]};
            double c1[3] = {c0[0] + G->w[0], c0[1] + G->w[1], c0[2] + G->w[2]};
            if (!dau_meets_cell(g, pv, c0, c1)) continue;
            long c = ((long)ix * G->n[1] + iy) * G->n[2] + iz;
            if (pass == 0) {
              cnt[c + 1]++;
              total++;
            } else {
              G->dau[cnt[c]++] = k;
            }
          }
    }
    if (pass == 0) {
      if (total > (1L << 28)) {
        free(cnt);
        return -1;
      }
      for (long c = 0; c < cells; c++) cnt[c + 1] += cnt[c];
      G->off = (int*)xcalloc((size_t)cells + 1, sizeof(int));
      G->dau = (int*)xcalloc((size_t)total, sizeof(int));
      memcpy(G->off, cnt, ((size_t)cells + 1) * sizeof(int));
    }
  }
  free(cnt);
  return 0;
}

/* Switch the voxel mode on (building the grids once) or off.  0 on success. */
int og_set_voxels(og_geom* g, int on) {
  if (on && !g->vgrid) {
    g->vgrid = (og_vgrid*)xcalloc(g->n_lv, sizeof(og_vgrid));
    for (int l = 0; l < g->n_lv; l++) {
      if (g->lv_dau_cnt[l] >= 4 && build_grid(g, l, &g->vgrid[l]) != 0) {
        og_free_voxels(g);
        return -1;
      }
    }
  }
  g->use_voxels = on;
  return 0;
}

static const og_vgrid* grid_of(const og_geom* g, int lv) {
  if (!g->use_voxels || !g->vgrid || !g->vgrid[lv].off) return NULL;
  return &g->vgrid[lv];
}

static int cell_index(const og_vgrid* G, int i, double x) {
  double a = floor((x - G->lo[i]) / G->w[i]);
  return a < 0 ? 0 : (a > G->n[i] - 1 ? G->n[i] - 1 : (int)a);
}

/* Descend from touchable T (assumed to hold the point) into the deepest
 * daughter that holds it; daughters are tried in index order and the first
 * match wins.  `blocked` is a slot skipped at the first level only. */
static int descend(const og_geom* g, int T, const double* pg, const double* vg, int blocked) {
  double pl[3], vl[3];
  frame_of(g, T, pg, vg, pl, vl);
  for (;;) {
    int lv = g->t_lv[T];
    int found = -1;
    double pd[3], vd[3];
    /* candidates: every slot, or the slots listed in the point's cell */
    const og_vgrid* G = grid_of(g, lv);
    const int* list = NULL;
    int n_cand = g->lv_dau_cnt[lv];
    if (G) {
      long c = ((long)cell_index(G, 0, pl[0]) * G->n[1] + cell_index(G, 1, pl[1])) * G->n[2] +
               cell_index(G, 2, pl[2]);
      list = G->dau + G->off[c];
      n_cand = G->off[c + 1] - G->off[c];
    }
    for (int i = 0; i < n_cand; i++) {
      int k = list ? list[i] : i;
      if (k == blocked) continue;
      int pv = g->lv_dau_off[lv] + k;
      to_local(g->pv_rot + 9 * pv, g->pv_trans + 3 * pv, pl, pd);
      if (vg) dir_to_local(g->pv_rot + 9 * pv, vl, vd);
      if (og_solid_inside(lv_solid_of(g, g->pv_lv[pv]), pd, vg ? vd : NULL) == OG_IN) {
        found = k;
        break;
      }
    }
    if (found < 0) return T;
    int pv = g->lv_dau_off[lv] + found;
    T = g->t_child_base[T] + found;
    to_local(g->pv_rot + 9 * pv, g->pv_trans + 3 * pv, pl, pd);
    memcpy(pl, pd, sizeof(pd));
    if (vg) {
      dir_to_local(g->pv_rot + 9 * pv, vl, vd);
      memcpy(vl, vd, sizeof(vd));
    }
    blocked = -1;
  }
}

/* LocateGlobalPoint: the deepest touchable holding pg (-1: outside the world). */
static int locate(const og_geom* g, const double* pg, const double* vg) {
  if (og_solid_inside(lv_solid_of(g, g->world_lv), pg, vg) == OG_OUT) return -1;
  return descend(g, 0, pg, vg, -1);
}

/* ComputeStep by brute force: the mother's exit distance against every
 * daughter's entry distance; the mother wins ties, then the lowest slot. */
static double compute_step_voxels(const og_geom* g, const og_vgrid* G, int lv, const double* pl,
                                  const double* vl, int* lim);

static double compute_step(const og_geom* g, int T, const double* pg, const double* vg, int* lim) {
  double pl[3], vl[3];
  frame_of(g, T, pg, vg, pl, vl);
  int lv = g->t_lv[T];
  const og_vgrid* G = grid_of(g, lv);
  if (G) return compute_step_voxels(g, G, lv, pl, vl, lim);
  double s = og_solid_dist_out(lv_solid_of(g, lv), pl, vl);
  double second = kInf; /* next smallest distance, for the selection's margin */
  *lim = OG_LIM_MOTHER;
  for (int k = 0; k < g->lv_dau_cnt[lv]; k++) {
    int pv = g->lv_dau_off[lv] + k;
    double pd[3], vd[3];
    to_local(g->pv_rot + 9 * pv, g->pv_trans + 3 * pv, pl, pd);
    dir_to_local(g->pv_rot + 9 * pv, vl, vd);
    double t = og_solid_dist_in(lv_solid_of(g, g->pv_lv[pv]), pd, vd);
    if (t < s) {
      second = s;
      s = t;
      *lim = k;
    } else if (t < second) {
      second = t;
    }
  }
  if (second < kInf) NOTE_LEN(s, second);
  return s;
}

/* ComputeStep through the grid: the cells along the ray in order (a 3D DDA),
 * each daughter evaluated once; the walk stops once the best distance does
 * not exceed the current cell's exit, since a daughter not listed so far is
 * entered only beyond it.  The same minimum and tie rule as brute force: the
 * mother beats a daughter at equal distance, then the lowest slot. */
static double compute_step_voxels(const og_geom* g, const og_vgrid* G, int lv, const double* pl,
                                  const double* vl, int* lim) {
  double s = og_solid_dist_out(lv_solid_of(g, lv), pl, vl);
  *lim = OG_LIM_MOTHER;
  int nd = g->lv_dau_cnt[lv];
  unsigned char seen_small[512];
  unsigned char* seen = nd <= 512 ? seen_small : (unsigned char*)xcalloc(nd, 1);
  memset(seen, 0, nd <= 512 ? (size_t)nd : 0);
  int c[3], step[3];
  double tnext[3], dt[3];
  for (int i = 0; i < 3; i++) {
    c[i] = cell_index(G, i, pl[i]);
    if (vl[i] > 0) {
      step[i] = 1;
      tnext[i] = (G->lo[i] + (c[i] + 1) * G->w[i] - pl[i]) / vl[i];
      dt[i] = G->w[i] / vl[i];
    } else if (vl[i] < 0) {
      step[i] = -1;
      tnext[i] = (G->lo[i] + c[i] * G->w[i] - pl[i]) / vl[i];
      dt[i] = -G->w[i] / vl[i];
    } else {
      step[i] = 0;
      tnext[i] = kInf;
      dt[i] = kInf;
    }
  }
  for (;;) {
    long cell = ((long)c[0] * G->n[1] + c[1]) * G->n[2] + c[2];
    for (int i = G->off[cell]; i < G->off[cell + 1]; i++) {
      int k = G->dau[i];
      if (seen[k]) continue;
      seen[k] = 1;
      int pv = g->lv_dau_off[lv] + k;
      double pd[3], vd[3];
      to_local(g->pv_rot + 9 * pv, g->pv_trans + 3 * pv, pl, pd);
      dir_to_local(g->pv_rot + 9 * pv, vl, vd);
      double t = og_solid_dist_in(lv_solid_of(g, g->pv_lv[pv]), pd, vd);
      if (t < s || (t == s && *lim >= 0 && k < *lim)) {
        s = t;
        *lim = k;
      }
    }
    int ax = 0;
    if (tnext[1] < tnext[ax]) ax = 1;
    if (tnext[2] < tnext[ax]) ax = 2;
    double t_exit = tnext[ax];
    if (s <= t_exit) break;
    c[ax] += step[ax];
    if (c[ax] < 0 || c[ax] >= G->n[ax]) break; /* left the grid: every candidate seen */
    tnext[ax] += dt[ax];
  }
  if (seen != seen_small) free(seen);
  return s;
}

/* ComputeSafety by brute force: a lower bound on the isotropic distance to
 * the nearest boundary (mother or any daughter). */
static double compute_safety(const og_geom* g, int T, const double* pg) {
  double pl[3];
  frame_of(g, T, pg, NULL, pl, NULL);
  int lv = g->t_lv[T];
  double s = og_solid_safety_out(lv_solid_of(g, lv), pl);
  for (int k = 0; k < g->lv_dau_cnt[lv]; k++) {
    int pv = g->lv_dau_off[lv] + k;
    double pd[3];
    to_local(g->pv_rot + 9 * pv, g->pv_trans + 3 * pv, pl, pd);
    s = min2(s, og_solid_safety_in(lv_solid_of(g, g->pv_lv[pv]), pd));
  }
  return s;
}

/* Relocation after a geometry-limited step.  Entering daughter `lim`: step
 * into it and descend.  Leaving the mother: climb while the point is
 * outside the parent (or on its surface moving out), then search the
 * parent's daughters with the volume just left excluded. */
static int relocate(const og_geom* g, int T, const double* pg, const double* vg, int lim) {
  if (lim >= 0) return descend(g, g->t_child_base[T] + lim, pg, vg, -1);
  int left = T;
  int P = g->t_parent[T];
  while (P >= 0) {
    double pl[3], vl[3];
    frame_of(g, P, pg, vg, pl, vl);
    if (og_solid_inside(lv_solid_of(g, g->t_lv[P]), pl, vl) != OG_OUT) break;
    left = P;
    P = g->t_parent[P];
  }
  if (P < 0) return -1;
  return descend(g, P, pg, vg, g->t_slot[left]);
}

/* ------------------------------------------------------------------------ */
/* Query entry points (arrays of n queries).                                */
/* ------------------------------------------------------------------------ */

void og_locate(const og_geom* g, int n, const double* pos, const double* dir, int* out) {
  for (int i = 0; i < n; i++) out[i] = locate(g, pos + 3 * i, dir ? dir + 3 * i : NULL);
}

void og_compute_step(const og_geom* g, int n, const double* pos, const double* dir, const int* touch,
                     double* step, int* lim, int* next) {
  for (int i = 0; i < n; i++) {
    const double* p = pos + 3 * i;
    const double* v = dir + 3 * i;
    int T = touch ? touch[i] : locate(g, p, v);
    if (T < 0) {
      step[i] = kInf;
      lim[i] = OG_LIM_MOTHER;
      if (next) next[i] = -1;
      continue;
    }
    int l;
    double s = compute_step(g, T, p, v, &l);
    step[i] = s;
    lim[i] = l;
    if (next) {
      double q[3] = {p[0] + s * v[0], p[1] + s * v[1], p[2] + s * v[2]};
      next[i] = (s < kInf) ? relocate(g, T, q, v, l) : -1;
    }
  }
}

/* A direction in the frame of touchable T back to the global frame: the
 * placement rotations applied level by level from T up to the world. */
static void dir_to_global(const og_geom* g, int T, const double* vl, double* vg) {
  double v[3] = {vl[0], vl[1], vl[2]};
  for (int u = T; u > 0; u = g->t_parent[u]) {
    const double* R = g->pv_rot + 9 * g->t_pv[u];
    double w[3];
    for (int i = 0; i < 3; i++) w[i] = R[3 * i] * v[0] + R[3 * i + 1] * v[1] + R[3 * i + 2] * v[2];
    memcpy(v, w, sizeof(w));
  }
  memcpy(vg, v, sizeof(v));
}

/* ComputeStep with the exit normal at the end point: the outward normal of
 * the mother when the mother limits the step, the inward normal of the
 * entered daughter otherwise (both point along the direction of travel), in
 * the global frame.  valid: 0 no boundary reached, 1 a face, 2 an edge or a
 * corner (two or more faces within the tolerance). */
void og_compute_step_normal(const og_geom* g, int n, const double* pos, const double* dir, const int* touch,
                            double* step, int* lim, int* next, double* normal, int* valid) {
  og_compute_step(g, n, pos, dir, touch, step, lim, next);
  for (int i = 0; i < n; i++) {
    const double* p = pos + 3 * i;
    const double* v = dir + 3 * i;
    double* nv = normal + 3 * i;
    nv[0] = nv[1] = nv[2] = 0.0;
    valid[i] = 0;
    if (!(step[i] < kInf)) continue;
    int T = touch ? touch[i] : locate(g, p, v);
    if (T < 0) continue;
    int S = lim[i] >= 0 ? g->t_child_base[T] + lim[i] : T;
    double q[3] = {p[0] + step[i] * v[0], p[1] + step[i] * v[1], p[2] + step[i] * v[2]};
    double ql[3], nl[3];
    frame_of(g, S, q, NULL, ql, NULL);
    int faces = og_solid_normal(lv_solid_of(g, g->t_lv[S]), ql, nl);
    if (lim[i] >= 0)
      for (int k = 0; k < 3; k++) nl[k] = -nl[k];
    dir_to_global(g, S, nl, nv);
    valid[i] = faces > 1 ? 2 : 1;
  }
}

void og_compute_safety(const og_geom* g, int n, const double* pos, const int* touch, double* out) {
  for (int i = 0; i < n; i++) {
    const double* p = pos + 3 * i;
    int T = touch ? touch[i] : locate(g, p, NULL);
    out[i] = T < 0 ? 0.0 : compute_safety(g, T, p);
  }
}

/* Outward normals of one solid at n points (face counts in faces). */
int og_solid_normal_n(int type, const double* par, int n, const double* p, double* normals, int* faces) {
  og_solid s;
  if (solid_init(&s, type, par) != 0) return -1;
  for (int i = 0; i < n; i++) faces[i] = og_solid_normal(&s, p + 3 * i, normals + 3 * i);
  return 0;
}

/* Per-solid entry points for unit tests: op 0 d, 1 inside(p[,v]), 2 dist_in,
 * 3 dist_out, 4 safety_in, 5 safety_out. */
int og_solid_eval(int type, const double* par, int op, int n, const double* p, const double* v,
                  double* out) {
  og_solid s;
  if (solid_init(&s, type, par) != 0) return -1;
  for (int i = 0; i < n; i++) {
    const double* pp = p + 3 * i;
    const double* vv = v ? v + 3 * i : NULL;
    switch (op) {
      case 0: out[i] = og_solid_d(&s, pp); break;
      case 1: out[i] = og_solid_inside(&s, pp, vv); break;
      case 2: out[i] = og_solid_dist_in(&s, pp, vv); break;
      case 3: out[i] = og_solid_dist_out(&s, pp, vv); break;
      case 4: out[i] = og_solid_safety_in(&s, pp); break;
      case 5: out[i] = og_solid_safety_out(&s, pp); break;
      default: return -1;
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Alg. 1 (Sec. 3.1): free path length of one photon for a given Y.         */
/* ------------------------------------------------------------------------ */

/* Walk the ray boundary to boundary; S accumulates (t_j - t_{j-1}) mu_j and
 * the interaction lies at t_{j-1} + (Y - S_{j-1}) / mu_j.  Returns +inf when
 * the photon leaves the world first.  mu is the total attenuation of the
 * material at energy E. */
double og_free_path(const og_geom* g, const double* x0, const double* w, double E, double Y,
                    int* n_bounds) {
  double x[3] = {x0[0], x0[1], x0[2]};
  int T = locate(g, x, w);
  double t_prev = 0.0, S_prev = 0.0;
  int nb = 0;
  while (T >= 0) {
    double mu3[3];
    mu_lookup(g, g->lv_mat[g->t_lv[T]], E, mu3);
    double mu = mu3[0] + mu3[1] + mu3[2];
    int lim;
    double s = compute_step(g, T, x, w, &lim);
    double S = (mu > 0) ? S_prev + s * mu : S_prev;
    if (mu > 0 && S >= Y) {
      if (n_bounds) *n_bounds = nb;
      return t_prev + (Y - S_prev) / mu;
    }
    for (int i = 0; i < 3; i++) x[i] = x[i] + s * w[i];
    t_prev = t_prev + s;
    S_prev = S;
    T = relocate(g, T, x, w, lim);
    nb++;
    if (nb > 1000000) break;
  }
  if (n_bounds) *n_bounds = nb;
  return kInf;
}

/* ------------------------------------------------------------------------ */
/* Photon interactions.                                                      */
/* ------------------------------------------------------------------------ */

/* Klein-Nishina sampling of eps = E'/E by the Butcher-Messel mixture
 * (1960): branch 1 with weight ln(1+2k) samples 1/eps, branch 2 with weight
 * (1 - eps0^2)/2 samples eps; accept with 1 - eps sin^2/(1 + eps^2).
 * Three draws per trial in the order branch, value, acceptance. */
static void compton_sample(double E, og_stream* rs, double* eps_out, double* cost_out, double* sin2_out) {
  double k = E / kMe;
  double eps0 = 1.0 / (1.0 + 2.0 * k);
  double eps0sq = eps0 * eps0;
  double a1 = log(1.0 + 2.0 * k);
  double a2 = 0.5 * (1.0 - eps0sq);
  double eps = 1.0, onecost = 0.0, sint2 = 0.0;
  for (int trial = 0; trial < OG_MAX_COMPTON_TRIALS; trial++) {
    double r1 = og_next(rs), r2 = og_next(rs), r3 = og_next(rs);
    double epssq;
    note(r1 * (a1 + a2), a1, a1 + a2);
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
    note(r3, g, 1.0);
    if (r3 <= g) break;
  }
  *eps_out = eps;
  *cost_out = 1.0 - onecost;
  *sin2_out = sint2;
}

/* Rotate unit vector v by polar angle (cos, sin) and azimuth phi about v. */
static void rotate_dir(double* v, double cost, double sint, double phi) {
  double a = v[0], b = v[1], c = v[2];
  double cp = cos(phi), sp = sin(phi);
  double rp = sqrt(a * a + b * b);
  double n[3];
  note(rp, 1e-12, 1.0);
  if (rp < 1e-12) {
    n[0] = sint * cp;
    n[1] = sint * sp;
    n[2] = (c >= 0 ? 1.0 : -1.0) * cost;
  } else {
    double e1[3] = {a * c / rp, b * c / rp, -(a * a + b * b) / rp};
    double e2[3] = {-b / rp, a / rp, 0.0};
    for (int i = 0; i < 3; i++) n[i] = cost * v[i] + sint * (cp * e1[i] + sp * e2[i]);
  }
  double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  for (int i = 0; i < 3; i++) v[i] = n[i] / nn;
}

void og_compton_sample_n(double E, int n, uint64_t seed, double* eps, double* cost, int* draws) {
  for (int i = 0; i < n; i++) {
    og_stream rs = {seed, 0u, (uint32_t)i, 0u};
    double s2;
    compton_sample(E, &rs, &eps[i], &cost[i], &s2);
    if (draws) draws[i] = (int)rs.draw;
  }
}

void og_rotate(int n, double* v, const double* cost, const double* phi) {
  for (int i = 0; i < n; i++) {
    double st = sqrt((1.0 - cost[i]) * (1.0 + cost[i]));
    rotate_dir(v + 3 * i, cost[i], st, phi[i]);
  }
}

/* ------------------------------------------------------------------------ */
/* Transport.                                                                */
/* ------------------------------------------------------------------------ */

typedef struct {
  int32_t touchable, code;
  double step, edep, energy;
} og_logrec; /* 32 bytes */

/* Per-track summary: 64-bit FNV-1a (Fowler, Noll, Vo) over the touchable and
 * code of every record, each as four little-endian bytes, in record order;
 * the record count and fate; the sums of the records' steps and deposits. */
typedef struct {
  uint64_t hash;
  int32_t n, fate;
  double sum_step, sum_edep;
} og_digest; /* 32 bytes */

static uint64_t fnv1a_int32(uint64_t h, int32_t x) {
  uint32_t u = (uint32_t)x;
  for (int b = 0; b < 4; b++) {
    h ^= (u >> (8 * b)) & 0xffu;
    h *= 1099511628211ull;
  }
  return h;
}

typedef struct {
  const og_geom* g;
  uint64_t seed;
  double ecut;
  int64_t max_steps;
  double* edep_t;
  double* edep_ev;
  double* esc_ev;
  uint64_t* counters;
  og_logrec* log;
  int64_t log_cap;
  int32_t* log_n;
  int32_t* log_fate;
  double* start; /* optional [3 n][7]: position, direction and energy at each track's start */
  og_digest* digest; /* optional [3 n] */
  float* margin;     /* optional [3 n][log_cap]: smallest decision margin behind each record */
  float* tail;       /* optional [3 n]: smallest margin after the last record */
} og_run;

static void log_step(og_run* r, int64_t slot, int64_t* nrec, int T, int code, double step, double edep,
                     double energy) {
  if (r->digest) {
    og_digest* d = r->digest + slot;
    d->hash = fnv1a_int32(fnv1a_int32(d->hash, T), code);
    d->sum_step += step;
    d->sum_edep += edep;
  }
  if (r->margin && *nrec < r->log_cap) r->margin[slot * r->log_cap + *nrec] = (float)og_margin;
  og_margin = INFINITY;
  if (r->log && *nrec < r->log_cap) {
    og_logrec* q = r->log + slot * r->log_cap + *nrec;
    q->touchable = T;
    q->code = code;
    q->step = step;
    q->edep = edep;
    q->energy = energy;
  }
  (*nrec)++;
}

/* One photon history (Alg. 1 repeated after every interaction).  Pair
 * production ends the track and hands back two annihilation photons. */
static int track(og_run* r, uint32_t event, uint32_t key, int64_t slot, double* x, double* v, double E,
                 double* pair_x, double* pair_w) {
  const og_geom* g = r->g;
  og_stream rs = {r->seed, event, key, 0u};
  int64_t nrec = 0;
  int fate;
  r->counters[OG_C_TRACKS]++;
  og_margin = INFINITY;
  if (r->digest) {
    og_digest* d = r->digest + slot;
    d->hash = 14695981039346656037ull;
    d->n = 0;
    d->fate = 0;
    d->sum_step = 0.0;
    d->sum_edep = 0.0;
  }
  if (r->start) {
    double* q = r->start + 7 * slot;
    for (int i = 0; i < 3; i++) {
      q[i] = x[i];
      q[3 + i] = v[i];
    }
    q[6] = E;
  }
  int T = locate(g, x, v);
  if (T < 0) {
    r->esc_ev[event] += E;
    r->counters[OG_C_ESCAPED]++;
    fate = OG_FATE_ESCAPED;
    goto done;
  }
  double nl = -log(og_next(&rs));
  int zero = 0;
  int64_t steps = 0;
  for (;;) {
    note(E, r->ecut, E);
    if (E < r->ecut) {
      r->edep_t[T] += E;
      r->edep_ev[event] += E;
      r->counters[OG_C_CUTOFF]++;
      fate = OG_FATE_CUTOFF;
      goto done;
    }
    if (steps >= r->max_steps) {
      r->counters[OG_C_TRUNCATED]++;
      fate = OG_FATE_TRUNCATED;
      goto done;
    }
    double mu3[3];
    mu_lookup(g, g->lv_mat[g->t_lv[T]], E, mu3);
    double mu = mu3[0] + mu3[1] + mu3[2];
    double s_phys = mu > 0 ? nl / mu : kInf;
    int lim;
    double s_geo = compute_step(g, T, x, v, &lim);
    steps++;
    r->counters[OG_C_STEPS]++;
    if (s_phys < kInf) note(s_phys, s_geo, max2(og_scale, max2(s_phys, s_geo)));
    if (s_phys <= s_geo) {
      /* the interaction point of Alg. 1: T = t_{j-1} + (Y - S_{j-1}) / mu_j */
      for (int i = 0; i < 3; i++) x[i] = x[i] + s_phys * v[i];
      zero = 0;
      double u = og_next(&rs) * mu;
      note(u, mu3[0], mu);
      note(u, mu3[0] + mu3[1], mu);
      if (u < mu3[0]) {
        r->edep_t[T] += E;
        r->edep_ev[event] += E;
        r->counters[OG_C_PE]++;
        log_step(r, slot, &nrec, T, OG_LIM_PE, s_phys, E, 0.0);
        fate = OG_FATE_ABSORBED;
        goto done;
      } else if (u < mu3[0] + mu3[1]) {
        double eps, cost, sin2;
        compton_sample(E, &rs, &eps, &cost, &sin2);
        double phi = 2.0 * M_PI * og_next(&rs);
        rotate_dir(v, cost, sqrt(sin2), phi);
        double dep = E * (1.0 - eps);
        E = eps * E;
        r->edep_t[T] += dep;
        r->edep_ev[event] += dep;
        r->counters[OG_C_COMPTON]++;
        log_step(r, slot, &nrec, T, OG_LIM_COMPTON, s_phys, dep, E);
      } else {
        double dep = E - 2.0 * kMe;
        r->edep_t[T] += dep;
        r->edep_ev[event] += dep;
        r->counters[OG_C_PAIR]++;
        double u1 = og_next(&rs), u2 = og_next(&rs);
        double ct = 1.0 - 2.0 * u1;
        double st = 2.0 * sqrt(u1 * (1.0 - u1));
        double ph = 2.0 * M_PI * u2;
        pair_w[0] = st * cos(ph);
        pair_w[1] = st * sin(ph);
        pair_w[2] = ct;
        for (int i = 0; i < 3; i++) pair_x[i] = x[i];
        log_step(r, slot, &nrec, T, OG_LIM_PAIR, s_phys, dep, 0.0);
        fate = OG_FATE_PAIR;
        goto done;
      }
      nl = -log(og_next(&rs));
    } else {
      /* Eq. 6: the optical depth spent on this segment */
      for (int i = 0; i < 3; i++) x[i] = x[i] + s_geo * v[i];
      if (mu > 0) {
        nl = nl - s_geo * mu;
        if (nl < 0) nl = 0;
      }
      log_step(r, slot, &nrec, T, lim, s_geo, 0.0, E);
      r->counters[OG_C_CROSSINGS]++;
      NOTE_LEN(s_geo, kTol);
      if (s_geo < kTol) zero++;
      else zero = 0;
      if (zero >= OG_ZERO_KILL) {
        r->edep_t[T] += E;
        r->edep_ev[event] += E;
        r->counters[OG_C_STUCK]++;
        fate = OG_FATE_STUCK;
        goto done;
      }
      if (zero > 0 && zero % OG_ZERO_PUSH == 0) {
        for (int i = 0; i < 3; i++) x[i] = x[i] + 100.0 * kTol * v[i];
        r->counters[OG_C_PUSHES]++;
      }
      T = relocate(g, T, x, v, lim);
      if (T < 0) {
        r->esc_ev[event] += E;
        r->counters[OG_C_ESCAPED]++;
        fate = OG_FATE_ESCAPED;
        goto done;
      }
    }
  }
done:
  if (r->log_n) r->log_n[slot] = (int32_t)(nrec > 0x7fffffff ? 0x7fffffff : nrec);
  if (r->log_fate) r->log_fate[slot] = fate;
  if (r->digest) {
    r->digest[slot].n = (int32_t)(nrec > 0x7fffffff ? 0x7fffffff : nrec);
    r->digest[slot].fate = fate;
  }
  if (r->tail) r->tail[slot] = (float)og_margin;
  return fate;
}

/* Transport n primaries.  Outputs are accumulated (caller zeroes them).
 * Logs, when given, hold log_cap records for each of 3 n track slots:
 * slot 3i is primary i, 3i+1 and 3i+2 its annihilation photons. */
int og_transport(const og_geom* g, int64_t n, const int32_t* event, const int32_t* prim_id,
                 const double* pos, const double* dir, const double* energy, uint64_t seed, double ecut,
                 int64_t max_steps, double* edep_t, double* edep_ev, double* esc_ev, uint64_t* counters,
                 og_logrec* log, int64_t log_cap, int32_t* log_n, int32_t* log_fate, double* start,
                 og_digest* digest, float* margin, float* tail) {
  og_run r = {g,       seed,     ecut,  max_steps, edep_t, edep_ev, esc_ev, counters, log, log_cap,
              log_n,   log_fate, start, digest,    margin, tail};
  /* coordinate scale of the margins: the world's largest extent */
  {
    const og_solid* w = lv_solid_of(g, g->world_lv);
    double e = w->par[0];
    if (w->type == OG_BOX) e = max2(w->par[0], max2(w->par[1], w->par[2]));
    else if (w->type == OG_TRD) e = max2(max2(max2(w->par[0], w->par[1]), max2(w->par[2], w->par[3])), w->par[4]);
    else if (w->type == OG_SPHERE) e = w->par[1];
    else if (w->type != OG_ORB) e = max2(w->Ao + fabs(w->Bo) * w->dz, w->dz);
    og_scale = max2(1.0, e);
  }
  og_margin_on = (margin || tail) ? 1 : 0;
  for (int64_t i = 0; i < n; i++) {
    double x[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
    double v[3] = {dir[3 * i], dir[3 * i + 1], dir[3 * i + 2]};
    uint32_t key = ((uint32_t)prim_id[i]) << 2;
    double px[3], pw[3];
    int fate = track(&r, (uint32_t)event[i], key, 3 * i, x, v, energy[i], px, pw);
    if (fate == OG_FATE_PAIR) {
      /* two annihilation photons at the conversion point, back to back */
      double dx[3], dw[3];
      double x1[3] = {px[0], px[1], px[2]}, w1[3] = {pw[0], pw[1], pw[2]};
      track(&r, (uint32_t)event[i], key | 1u, 3 * i + 1, x1, w1, kMe, dx, dw);
      double x2[3] = {px[0], px[1], px[2]}, w2[3] = {-pw[0], -pw[1], -pw[2]};
      track(&r, (uint32_t)event[i], key | 2u, 3 * i + 2, x2, w2, kMe, dx, dw);
    }
  }
  og_margin_on = 0;
  return 0;
}

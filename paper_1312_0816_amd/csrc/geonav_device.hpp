// Device-side records and per-lane shape algorithms of libgeonav (gfx950, FP64).
//
// One lane evaluates one track. Every algorithm is branch-free over lanes:
// all candidate surfaces of a shape are evaluated and the valid smallest one
// is kept with selects, so a wavefront never diverges inside a shape. The
// only branches are on the shape kind and the hole and convexity flags,
// which are uniform across a wavefront where the daughters are walked in
// lockstep (shape queries, sequential navigator loops); in a batch of the
// compacted navigators the lanes hold different daughters, and lanes of
// each kind take that kind's code in turn.
//
// Each distance query is a minimum over per-surface candidates (faces,
// z-planes, the outer and inner cylinder/cone nappes): for DistFromOutside
// a candidate is a point where the line enters the solid through that
// surface; for DistFromInside it is the first crossing of that surface's
// constraint. Quadric roots use the cancellation-free pair of formulas
// (numerator and denominator chosen by the sign of B), one division each.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gn {

constexpr double kBig = 1e30;
constexpr int kMaxDaughters = 1024;  // daughters per volume (GEO_MAX_DAUGHTERS)
constexpr int kCensusSlots = 16, kCensusCull = 14, kCensusTracks = 15;
// kPcon is an uncut polycone, kPcons one cut to an azimuth range.
enum : int32_t { kBox = 0, kTube = 1, kCone = 2, kTubs = 3, kCons = 4, kPcon = 5, kPcons = 6 };

// Shape with host-derived constants.
//   BOX  c0..2 = dx, dy, dz
//   TUBE c0 = rmin, c1 = rmax, c2 = dz, c3 = rmin^2, c4 = rmax^2
//   CONE c0 = dz, radius r(z) = a + b z: c1 = a_out, c2 = b_out, c3 = a_in, c4 = b_in,
//        c5..8 = rmin1, rmax1, rmin2, rmax2, c9..12 = their squares,
//        c13 = 1/sqrt(1 + b_out^2), c14 = 1/sqrt(1 + b_in^2),
//        c15 = 1/|outer edge|^2, c16 = 1/|inner edge|^2 (profile edges in (r, z))
//   TUBS, CONS (segments: the tube or cone cut to the azimuths [phi1, phi2],
//        phi2 = phi1 + dphi < phi1 + 2 pi, axis included): the base kind's
//        constants, and c17, c18 = cos phi1, sin phi1; c19, c20 = cos phi2, sin phi2.
//   PCON, PCONS (polycone, uncut or cut): its sections live in a PconRec
//        (see below); PCONS keeps the azimuth range in c17..c20.
// Slack of the range tests at candidate hit points (see "Edges" below):
//   c21 = eps = 1e-12 x the shape's bounding radius, and the limits widened
//   by it: BOX c3..5 = dx, dy, dz + eps; TUBE/TUBS c5 = dz + eps,
//   c6, c7 = (rmin - eps)^2 (0 if rmin <= eps), (rmax + eps)^2; CONE/CONS
//   c22 = dz + eps, c23..26 = the same two squares at -dz and at +dz.
struct alignas(16) ShapeRec {
    int32_t kind;
    int32_t hole;    // tube/cone: an inner surface exists (not both inner radii 0)
    int32_t convex;  // segment: dphi <= pi (the azimuth range is convex)
    int32_t pad;
    double c[28];
};
static_assert(sizeof(ShapeRec) == 240, "ShapeRec layout");

// Polycone: nz planes z_0 < ... < z_{nz-1} (nz <= kPconMax) with radii
// rin/rout at each; between two planes the radii are linear in z, section
// j's nappes being r = ao[j] + bo[j] z (outer) and ai[j] + bi[j] z (inner,
// present when bit j of hole_mask is set: not both inner radii 0).
constexpr int kPconMax = 8;
// The daughter and culling tables hold each volume's records padded to a
// multiple of kCullChunk; padding records have q (culling record) and
// cull_r2 (daughter record) = -infinity, so that
// no culling test passes them.
constexpr int kCullChunk = 4;
struct alignas(16) PconRec {
    int32_t nz;
    int32_t hole_mask;
    int32_t pad[2];
    double z[kPconMax], rin[kPconMax], rout[kPconMax];
    double rin2_0, rout2_0, rin2_l, rout2_l;  // squared end radii, widened by eps (hit tests)
    double ao[kPconMax - 1], bo[kPconMax - 1], ai[kPconMax - 1], bi[kPconMax - 1];
    double inv_eo[kPconMax - 1], inv_ei[kPconMax - 1];   // 1 / |profile edge|^2, outer and inner
    double eps;  // slack of the range tests at hit points: 1e-12 x (max |z| + max rmax)
    double pad2;
};
static_assert(sizeof(PconRec) == 592, "PconRec layout");

// A placed daughter: mother-frame point = R * local + T.
struct alignas(16) DaughterRec {
    double rot[9];   // R, row-major
    double tr[3];    // T
    double bound_r;  // radius of a sphere about the local origin holding the shape
    // the culling radius (bound_r enlarged by 1e-6 relative + 1e-6) squared
    // and itself, for the tests with offsets (which form w = p - T
    // explicitly) and the safety's reach; -infinity and 0 in padding records
    double cull_r2;
    double cull_r;
    const PconRec *pcon;  // the polycone's sections (device), or NULL
    ShapeRec shape;
};
static_assert(sizeof(DaughterRec) == 368, "DaughterRec layout");

// Culling record of a daughter, in its own compact array (32 B, so the
// records of a whole volume stay in the scalar cache during the daughter
// loop, and a chunk of four is 128 contiguous bytes, two scalar loads): the
// centre of the bounding sphere in the mother frame (T) and the threshold q
// of the expanded test of the compacted navigator: that test evaluates the
// squared distance from T to the track's half-line, less |T|^2, as
// |p|^2 - 2 p.T - b^2 with b = min((p - T).e, 0) and e = d / |d| (1 / |d|
// to a few ulp); every term is at most (|p| + |T|)^2, so the rounding error
// is below 16 eps (2 R + 2 |T|)^2 for a track inside the mother (R the
// mother's bounding radius); q = r2 - |T|^2 + 64 eps (3 R + 2 |T|)^2, r2
// the square of the culling radius. The radius itself and r2 sit in the
// daughter record.
struct alignas(16) CullRec {
    double tx, ty, tz, q;
};
static_assert(sizeof(CullRec) == 32, "CullRec layout");

struct alignas(16) VolumeRec {
    ShapeRec mother;
    int32_t nd;     // number of daughters
    int32_t first;  // index of daughter 0 in the daughter and culling tables
    const PconRec *pcon;  // the mother's polycone sections (device), or NULL
    double bound_r;       // radius of a sphere about the origin holding the mother
};
static_assert(sizeof(VolumeRec) == 272, "VolumeRec layout");

struct TracksDev {
    const double *x, *y, *z, *ux, *uy, *uz;
    int64_t n;
};

// Work unit of the batched kernel: `count` tracks of volume `volume` at
// pool index `offset`.
struct Tile {
    int32_t volume;
    int32_t count;
    int64_t offset;
};

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ double sq(double a) { return a * a; }

// n / d from the hardware reciprocal refined by two Newton steps: within
// about one ulp of the rounded quotient, six instructions instead of the
// eleven of the IEEE division sequence (which also rescales denormal and
// huge operands). A zero d gives NaN; every call site either has d in the
// normal range or rejects the result (the NaN fails its t >= 0 / ordering
// tests).
__device__ __forceinline__ double fdiv(double n, double d) {
    double r = __builtin_amdgcn_rcp(d);
    double e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    return n * r;
}

// 1 / sqrt(x) for finite x > 0, within a few ulp: the hardware estimate
// refined by two Newton steps (each squares the relative error, so an
// estimate within 2^-13 reaches full precision). x below 2^-960, subnormals
// included, is scaled by 2^1000 first.
__device__ __forceinline__ double rsqrt_fine(double x) {
    const bool tiny = x < 0x1p-960;
    const double xs = tiny ? x * 0x1p1000 : x;
    double z = __builtin_amdgcn_rsq(xs);
    double e = fma(-xs * z, z, 1.0);  // 1 - x z^2
    z = fma(0.5 * z, e, z);
    e = fma(-xs * z, z, 1.0);
    z = fma(0.5 * z, e, z);
    return tiny ? z * 0x1p500 : z;
}

// sqrt(x) from the hardware reciprocal square root with a Goldschmidt step
// and two corrections (within about one ulp; 11 instructions against 17 for
// the correctly rounded sequence). x below 1e-300 (including 0 and the
// clamped negative discriminants) gives 0: a tangent line, or a safety below
// 1e-150.
__device__ __forceinline__ double fsqrt(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    const double r = fma(-h, g, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    double d = fma(-g, g, x);
    g = fma(d, h, g);
    d = fma(-g, g, x);
    g = fma(d, h, g);
    return x > 1e-300 ? g : 0.0;
}

// Candidate update: keep the smallest valid t; on equal t the earlier
// candidate (lower surface id) stays.
__device__ __forceinline__ void take(bool ok, double t, int id, double &best, int &sid) {
    const bool better = ok && (t < best);
    best = better ? t : best;
    sid = better ? id : sid;
}

// Roots of f(t) = A t^2 + 2 B t + C, with s = sqrt(B^2 - A C).
// Root where f goes from + to - (A t + B = -s): (-B - s) / A = C / (s - B).
__device__ __forceinline__ double root_down(double A, double B, double C, double s) {
    const bool neg = B <= 0.0;
    const double num = neg ? C : -(B + s);
    const double den = neg ? (s - B) : A;
    return fdiv(num, den);
}
// Root where f goes from - to + (A t + B = +s): (-B + s) / A = -C / (s + B).
__device__ __forceinline__ double root_up(double A, double B, double C, double s) {
    const bool pos = B >= 0.0;
    const double num = pos ? -C : (s - B);
    const double den = pos ? (s + B) : A;
    return fdiv(num, den);
}

// Near-double roots. A line through a nappe's apex (or tangent to it) has a
// double root t0: B^2 - A C vanishes in exact arithmetic but comes out as
// +-(a few ulps of B^2), whose square root would move both roots by about
// sqrt(eps) t0. Within kSnap B^2 of zero the discriminant is taken as 0, and
// the formulas above then give t0 = C / (-B) = -B / A to rounding.
constexpr double kSnap = 64.0 * 2.220446049250313e-16;
__device__ __forceinline__ double disc_sqrt(double disc, double B) {
    return disc > kSnap * (B * B) ? fsqrt(disc) : 0.0;
}
__device__ __forceinline__ bool disc_ok(double disc, double B) { return disc >= -kSnap * (B * B); }

// Edges. A candidate counts only if its hit point lies on the surface's part
// that bounds the solid (a face's rectangle or annulus, a nappe's z range, a
// segment's azimuth range). At an edge two such tests meet, and a line
// through the edge could fail both by rounding. The tests at hit points
// therefore allow a slack eps of 1e-12 x the shape's size; a hit that far
// outside a face is within a comparable distance of the neighbouring
// surface's own hit. The membership tests themselves (Contains, and "the
// point is inside" in the distance queries) stay exact.

// ---------------------------------------------------------------------- box
__device__ __forceinline__ bool box_contains(const double *c, double x, double y, double z) {
    return fabs(x) <= c[0] && fabs(y) <= c[1] && fabs(z) <= c[2];
}

__device__ __forceinline__ double box_safety(const double *c, double x, double y, double z) {
    const double ex = fabs(x) - c[0], ey = fabs(y) - c[1], ez = fabs(z) - c[2];
    const double m = fmax(ex, fmax(ey, ez));
    const double ox = fmax(ex, 0.0), oy = fmax(ey, 0.0), oz = fmax(ez, 0.0);
    const double out = fsqrt(ox * ox + oy * oy + oz * oz);
    return m <= 0.0 ? -m : out;
}

// Entering face a: the point is beyond the slab (|p_a| > D_a) and moves
// towards it; the entry point must lie within the other two slabs.
__device__ __forceinline__ double box_dist_out(const double *c, double x, double y, double z,
                                               double ux, double uy, double uz, int &sid) {
    const double ax = fabs(x) - c[0], ay = fabs(y) - c[1], az = fabs(z) - c[2];
    const bool inside = ax <= 0.0 && ay <= 0.0 && az <= 0.0;
    double best = kBig;
    sid = -1;
    {
        const double t = fdiv(ax, fabs(ux));
        const bool ok = ax > 0.0 && x * ux < 0.0 && fabs(fma(t, uy, y)) <= c[4] &&
                        fabs(fma(t, uz, z)) <= c[5];
        take(ok, t, 0, best, sid);
    }
    {
        const double t = fdiv(ay, fabs(uy));
        const bool ok = ay > 0.0 && y * uy < 0.0 && fabs(fma(t, ux, x)) <= c[3] &&
                        fabs(fma(t, uz, z)) <= c[5];
        take(ok, t, 1, best, sid);
    }
    {
        const double t = fdiv(az, fabs(uz));
        const bool ok = az > 0.0 && z * uz < 0.0 && fabs(fma(t, ux, x)) <= c[3] &&
                        fabs(fma(t, uy, y)) <= c[4];
        take(ok, t, 2, best, sid);
    }
    return inside ? 0.0 : best;
}

// Leaving: the first face the line reaches on each axis.
// The same distance without the surface that sets it, for callers that only
// need the value: the three exits taken with fmin, which skips the NaN of an
// axis the direction does not move along (fdiv by 0); the result equals
// box_dist_in's bit for bit (the smallest exit below kBig, else kBig; 0
// outside).
__device__ __forceinline__ double box_exit(const double *c, double x, double y, double z, double ux,
                                           double uy, double uz) {
    const double tx = fdiv(c[0] - (ux > 0.0 ? x : -x), fabs(ux));
    const double ty = fdiv(c[1] - (uy > 0.0 ? y : -y), fabs(uy));
    const double tz = fdiv(c[2] - (uz > 0.0 ? z : -z), fabs(uz));
    const double best = fmin(kBig, fmin(tx, fmin(ty, tz)));
    return box_contains(c, x, y, z) ? best : 0.0;
}

__device__ __forceinline__ double box_dist_in(const double *c, double x, double y, double z,
                                              double ux, double uy, double uz, int &sid) {
    const bool inside = box_contains(c, x, y, z);
    double best = kBig;
    sid = -1;
    take(ux != 0.0, fdiv(c[0] - (ux > 0.0 ? x : -x), fabs(ux)), 0, best, sid);
    take(uy != 0.0, fdiv(c[1] - (uy > 0.0 ? y : -y), fabs(uy)), 1, best, sid);
    take(uz != 0.0, fdiv(c[2] - (uz > 0.0 ? z : -z), fabs(uz)), 2, best, sid);
    return inside ? best : 0.0;
}

// --------------------------------------------------------------------- tube
// Surfaces: 0 = z planes, 1 = outer cylinder, 2 = inner cylinder.
__device__ __forceinline__ bool tube_contains(const double *c, double x, double y, double z) {
    const double rsq = x * x + y * y;
    return fabs(z) <= c[2] && rsq <= c[4] && rsq >= c[3];
}

// (r, z) profile is the rectangle [rmin, rmax] x [-dz, dz]; without a hole
// the axis bounds no surface.
__device__ __forceinline__ double tube_safety(const double *c, int hole, double x, double y,
                                              double z) {
    const double r = fsqrt(x * x + y * y);
    const double eo = r - c[1];
    const double ei = hole ? c[0] - r : -kBig;
    const double ez = fabs(z) - c[2];
    const double er = fmax(eo, ei);
    const double m = fmax(er, ez);
    const double orr = fmax(er, 0.0), oz = fmax(ez, 0.0);
    const double out = fsqrt(orr * orr + oz * oz);
    return m <= 0.0 ? -m : out;
}

// ------------------------------------------------------------ azimuth range
// A segment keeps the azimuths [phi1, phi2] and the z axis. With the inward
// normals of its two bounding half-planes, n1 = (-sin phi1, cos phi1) and
// n2 = (sin phi2, -cos phi2), a point q is in the range when a = n1.q >= 0
// and b = n2.q >= 0 if dphi <= pi (a convex range), and when a >= 0 or
// b >= 0 if dphi > pi (the complement is then the open convex wedge a < 0,
// b < 0). a and b are the signed distances from the two face planes.
__device__ __forceinline__ double wedge_a(const double *c, double x, double y) {
    return fma(c[17], y, -c[18] * x);
}
__device__ __forceinline__ double wedge_b(const double *c, double x, double y) {
    return fma(c[20], x, -c[19] * y);
}
__device__ __forceinline__ bool wedge_in(const ShapeRec &s, double x, double y) {
    const double a = wedge_a(s.c, x, y), b = wedge_b(s.c, x, y);
    return s.convex ? (a >= 0.0 && b >= 0.0) : (a >= 0.0 || b >= 0.0);
}
// The same for a candidate's hit point, with the slack eps (c21).
__device__ __forceinline__ bool wedge_in_hit(const ShapeRec &s, double x, double y) {
    const double a = wedge_a(s.c, x, y), b = wedge_b(s.c, x, y);
    const double e = -s.c[21];
    return s.convex ? (a >= e && b >= e) : (a >= e || b >= e);
}

// Leaving the range along the line (the point is in it). Convex range: the
// first plane crossed outwards. Wider range: entering the open complement
// {a < 0} and {b < 0}, which happens at the later of the starts of the two
// half-lines {t : a(t) < 0}, {t : b(t) < 0}, provided neither has ended by
// then. Surfaces 3 and 4.
__device__ __forceinline__ void wedge_exit(const ShapeRec &s, double x, double y, double ux,
                                           double uy, double &best, int &sid) {
    const double a0 = wedge_a(s.c, x, y), da = wedge_a(s.c, ux, uy);
    const double b0 = wedge_b(s.c, x, y), db = wedge_b(s.c, ux, uy);
    const double ta = fdiv(-a0, da), tb = fdiv(-b0, db);
    if (s.convex) {
        take(da < 0.0, ta, 3, best, sid);
        take(db < 0.0, tb, 4, best, sid);
    } else {
        // {t : a(t) < 0} is (ta, inf) for da < 0, (-inf, ta) for da > 0, and
        // everything or nothing for da == 0
        const double lo_a = da < 0.0 ? ta : ((da > 0.0 || a0 < 0.0) ? -kBig : kBig);
        const double hi_a = da > 0.0 ? ta : ((da < 0.0 || a0 < 0.0) ? kBig : -kBig);
        const double lo_b = db < 0.0 ? tb : ((db > 0.0 || b0 < 0.0) ? -kBig : kBig);
        const double hi_b = db > 0.0 ? tb : ((db < 0.0 || b0 < 0.0) ? kBig : -kBig);
        const double lo = fmax(lo_a, lo_b), hi = fmin(hi_a, hi_b);
        take(lo < hi && hi > 0.0 && lo >= 0.0, lo, lo_a >= lo_b ? 3 : 4, best, sid);
    }
}

__device__ __forceinline__ bool cone_contains(const double *c, int hole, double x, double y,
                                              double z);
__device__ __forceinline__ bool pcon_contains(const PconRec &P, double x, double y, double z);
__device__ __forceinline__ bool pcon_contains_hit(const PconRec &P, double x, double y, double z);

template <int BASE>
__device__ __forceinline__ bool base_contains(const ShapeRec &s, const PconRec *pc, double x,
                                              double y, double z) {
    if (BASE == kTube) return tube_contains(s.c, x, y, z);
    if (BASE == kCone) return cone_contains(s.c, s.hole, x, y, z);
    return pcon_contains(*pc, x, y, z);
}

// Membership of a face entry's hit point in the base solid, with the slack
// eps on every bound.
template <int BASE>
__device__ __forceinline__ bool base_contains_hit(const ShapeRec &s, const PconRec *pc, double x,
                                                  double y, double z) {
    const double *c = s.c;
    const double rsq = x * x + y * y;
    if (BASE == kTube) return fabs(z) <= c[5] && rsq <= c[7] && rsq >= c[6];
    if (BASE == kCone) {
        const double wo = fma(c[2], z, c[1]) + c[21];
        const double wi = fmax(fma(c[4], z, c[3]) - c[21], 0.0);
        return fabs(z) <= c[22] && rsq <= wo * wo && rsq >= wi * wi;
    }
    return pcon_contains_hit(*pc, x, y, z);
}

// Entering the range through a flat face, at a point inside the base solid
// (surfaces 3 and 4). The line's parameters in the range follow from the
// half-lines {t : a(t) >= 0} and {t : b(t) >= 0}: for a convex range their
// intersection [w_lo, w_hi], entered at w_lo when the start is outside; for a
// wider range their union, the complement of the open interval in which the
// line crosses the wedge a < 0, b < 0, re-entered where that interval ends.
// Taking the entry from these intervals, not from a point test on each
// face's half-plane, keeps a line through the axis (both planes crossed at
// one point) exact.
template <int BASE>
__device__ __forceinline__ void face_entries(const ShapeRec &s, const PconRec *pc, double x,
                                             double y, double z, double ux, double uy, double uz,
                                             double &best, int &sid) {
    const double a0 = wedge_a(s.c, x, y), da = wedge_a(s.c, ux, uy);
    const double b0 = wedge_b(s.c, x, y), db = wedge_b(s.c, ux, uy);
    const double ta = fdiv(-a0, da), tb = fdiv(-b0, db);
    double t;
    bool ok;
    int id;
    if (s.convex) {
        // {a >= 0} is [ta, inf) for da > 0, (-inf, ta] for da < 0, all or nothing for da == 0
        const double lo_a = da > 0.0 ? ta : ((da < 0.0 || a0 >= 0.0) ? -kBig : kBig);
        const double hi_a = da < 0.0 ? ta : ((da > 0.0 || a0 >= 0.0) ? kBig : -kBig);
        const double lo_b = db > 0.0 ? tb : ((db < 0.0 || b0 >= 0.0) ? -kBig : kBig);
        const double hi_b = db < 0.0 ? tb : ((db > 0.0 || b0 >= 0.0) ? kBig : -kBig);
        t = fmax(lo_a, lo_b);
        ok = t <= fmin(hi_a, hi_b) && t >= 0.0;
        id = lo_a >= lo_b ? 3 : 4;
    } else {
        // {a < 0} is (ta, inf) for da < 0, (-inf, ta) for da > 0
        const double lo_a = da < 0.0 ? ta : ((da > 0.0 || a0 < 0.0) ? -kBig : kBig);
        const double hi_a = da > 0.0 ? ta : ((da < 0.0 || a0 < 0.0) ? kBig : -kBig);
        const double lo_b = db < 0.0 ? tb : ((db > 0.0 || b0 < 0.0) ? -kBig : kBig);
        const double hi_b = db > 0.0 ? tb : ((db < 0.0 || b0 < 0.0) ? kBig : -kBig);
        t = fmin(hi_a, hi_b);
        ok = fmax(lo_a, lo_b) < t && t >= 0.0 && t < kBig;
        id = hi_a <= hi_b ? 3 : 4;
    }
    const double xh = fma(t, ux, x), yh = fma(t, uy, y), zh = fma(t, uz, z);
    take(ok && base_contains_hit<BASE>(s, pc, xh, yh, zh), t, id, best, sid);
}

// With SEG (a segment) an entry through a base surface counts only at a hit
// point within the range, and the face entries join the candidates.
template <bool SEG>
__device__ __forceinline__ double tube_dist_out(const ShapeRec &S, double x, double y, double z,
                                                double ux, double uy, double uz, int &sid) {
    const double *c = S.c;
    const int hole = S.hole;
    const double dz = c[2];
    const double rsq = x * x + y * y;
    const bool inside = fabs(z) <= dz && rsq <= c[4] && rsq >= c[3] && (!SEG || wedge_in(S, x, y));
    double best = kBig;
    sid = -1;
    {   // z planes: from beyond the slab, moving towards it, landing on the annulus
        const double az = fabs(z) - dz;
        const double t = fdiv(az, fabs(uz));
        const double xh = fma(t, ux, x), yh = fma(t, uy, y);
        const double r2 = xh * xh + yh * yh;
        const bool ok = az > 0.0 && z * uz < 0.0 && r2 >= c[6] && r2 <= c[7] &&
                        (!SEG || wedge_in_hit(S, xh, yh));
        take(ok, t, 0, best, sid);
    }
    const double A = ux * ux + uy * uy;
    const double B = x * ux + y * uy;
    {   // outer cylinder, entered from r > rmax
        const double C = rsq - c[4];
        const double disc = B * B - A * C;
        const double s = disc_sqrt(disc, B);
        const double t = fdiv(C, s - B);
        const bool ok = C > 0.0 && B < 0.0 && disc_ok(disc, B) && fabs(fma(t, uz, z)) <= c[5] &&
                        (!SEG || wedge_in_hit(S, fma(t, ux, x), fma(t, uy, y)));
        take(ok, t, 1, best, sid);
    }
    if (hole) {  // inner cylinder, left from inside the hole into the material
        const double C = rsq - c[3];
        const double disc = B * B - A * C;
        const double s = disc_sqrt(disc, B);
        const double t = root_up(A, B, C, s);
        const bool ok = disc_ok(disc, B) && t >= 0.0 && fabs(fma(t, uz, z)) <= c[5] &&
                        (!SEG || wedge_in_hit(S, fma(t, ux, x), fma(t, uy, y)));
        take(ok, t, 2, best, sid);
    }
    if (SEG) face_entries<kTube>(S, nullptr, x, y, z, ux, uy, uz, best, sid);
    return inside ? 0.0 : best;
}

// With SEG the exit is the earlier of leaving the base and leaving the range.
template <bool SEG>
__device__ __forceinline__ double tube_dist_in(const ShapeRec &S, double x, double y, double z,
                                               double ux, double uy, double uz, int &sid) {
    const double *c = S.c;
    const int hole = S.hole;
    const double dz = c[2];
    const double rsq = x * x + y * y;
    const bool inside = fabs(z) <= dz && rsq <= c[4] && rsq >= c[3] && (!SEG || wedge_in(S, x, y));
    double best = kBig;
    sid = -1;
    take(uz != 0.0, fdiv(dz - (uz > 0.0 ? z : -z), fabs(uz)), 0, best, sid);
    const double A = ux * ux + uy * uy;
    const double B = x * ux + y * uy;
    {   // leave the outer cylinder
        const double C = rsq - c[4];
        const double disc = B * B - A * C;
        const double s = disc_sqrt(disc, B);
        const double t = root_up(A, B, C, s);
        take(disc_ok(disc, B) && t >= 0.0, t, 1, best, sid);
    }
    if (hole) {  // enter the hole's cylinder
        const double C = rsq - c[3];
        const double disc = B * B - A * C;
        const double s = disc_sqrt(disc, B);
        const double t = root_down(A, B, C, s);
        take(disc_ok(disc, B) && t >= 0.0, t, 2, best, sid);
    }
    if (SEG) wedge_exit(S, x, y, ux, uy, best, sid);
    return inside ? best : 0.0;
}

// --------------------------------------------------------------------- cone
// Surfaces: 0 = z planes, 1 = outer nappe r = a_out + b_out z,
// 2 = inner nappe r = a_in + b_in z. On a nappe, f = r^2 - (a + b z)^2 along
// the line is the quadratic A t^2 + 2 B t + C with
//   A = ux^2 + uy^2 - (b uz)^2, B = x ux + y uy - b uz w, C = x^2 + y^2 - w^2,
// w = a + b z. Its roots include the mirror nappe (a + b z < 0); a root on the
// mirror lies outside |z| <= dz (the radii are >= 0 on the slab), so the slab
// test at the root rejects it for entries, and for exits the z plane comes
// first.
__device__ __forceinline__ bool cone_contains(const double *c, int hole, double x, double y,
                                              double z) {
    const double rsq = x * x + y * y;
    const double wo = fma(c[2], z, c[1]);
    const double wi = fma(c[4], z, c[3]);
    return fabs(z) <= c[0] && rsq <= wo * wo && (!hole || rsq >= wi * wi);
}

__device__ __forceinline__ double seg_d2(double r, double z, double r0, double z0, double er,
                                         double ez, double inv_ee) {
    const double wr = r - r0, wz = z - z0;
    const double t = fmin(fmax((wr * er + wz * ez) * inv_ee, 0.0), 1.0);
    return sq(wr - t * er) + sq(wz - t * ez);
}

// Profile: trapezoid with corners (rmin1, -dz) (rmax1, -dz) (rmax2, dz)
// (rmin2, dz). Inside it is convex, so the distance is the smallest distance
// to the edges' lines; outside it is the smallest distance to the segments.
__device__ __forceinline__ double cone_safety(const double *c, int hole, double x, double y,
                                              double z) {
    const double dz = c[0];
    const double r = fsqrt(x * x + y * y);
    const double wo = fma(c[2], z, c[1]);
    const double wi = fma(c[4], z, c[3]);
    const bool inside = fabs(z) <= dz && r <= wo && (!hole || r >= wi);
    double din = fmin(dz - fabs(z), (wo - r) * c[13]);
    din = hole ? fmin(din, (r - wi) * c[14]) : din;
    // outside: bottom and top edges, outer and inner slanted edges
    const double rb = fmin(fmax(r, c[5]), c[6]);
    const double rt = fmin(fmax(r, c[7]), c[8]);
    double d2 = fmin(sq(r - rb) + sq(z + dz), sq(r - rt) + sq(z - dz));
    d2 = fmin(d2, seg_d2(r, z, c[6], -dz, c[8] - c[6], 2.0 * dz, c[15]));
    const double di2 = seg_d2(r, z, c[5], -dz, c[7] - c[5], 2.0 * dz, c[16]);
    d2 = hole ? fmin(d2, di2) : d2;
    return inside ? din : fsqrt(d2);
}

template <bool SEG>
__device__ __forceinline__ double cone_dist_out(const ShapeRec &S, double x, double y, double z,
                                                double ux, double uy, double uz, int &sid) {
    const double *c = S.c;
    const int hole = S.hole;
    const double dz = c[0];
    const double rsq = x * x + y * y;
    const double wo = fma(c[2], z, c[1]);
    const double wi = fma(c[4], z, c[3]);
    const bool inside = fabs(z) <= dz && rsq <= wo * wo && (!hole || rsq >= wi * wi) &&
                        (!SEG || wedge_in(S, x, y));
    double best = kBig;
    sid = -1;
    {   // z planes: the face's annulus depends on which end is hit
        const double az = fabs(z) - dz;
        const double t = fdiv(az, fabs(uz));
        const double xh = fma(t, ux, x), yh = fma(t, uy, y);
        const double r2 = xh * xh + yh * yh;
        // select between the two faces' verdicts (not their constants, which
        // stay uniform scalars)
        const bool on_bot = r2 >= c[23] && r2 <= c[24];
        const bool on_top = r2 >= c[25] && r2 <= c[26];
        const bool ok = az > 0.0 && z * uz < 0.0 && (z > 0.0 ? on_top : on_bot) &&
                        (!SEG || wedge_in_hit(S, xh, yh));
        take(ok, t, 0, best, sid);
    }
    const double A0 = ux * ux + uy * uy;
    const double B0 = x * ux + y * uy;
    {   // outer nappe: entered where f goes from + to -
        const double v = c[2] * uz;
        const double A = A0 - v * v, B = B0 - v * wo, C = rsq - wo * wo;
        const double disc = B * B - A * C;
        const double s = disc_sqrt(disc, B);
        const double t = root_down(A, B, C, s);
        const bool ok = disc_ok(disc, B) && t >= 0.0 && fabs(fma(t, uz, z)) <= c[22] &&
                        (!SEG || wedge_in_hit(S, fma(t, ux, x), fma(t, uy, y)));
        take(ok, t, 1, best, sid);
    }
    if (hole) {  // inner nappe: left from the hole where f goes from - to +
        const double v = c[4] * uz;
        const double A = A0 - v * v, B = B0 - v * wi, C = rsq - wi * wi;
        const double disc = B * B - A * C;
        const double s = disc_sqrt(disc, B);
        const double t = root_up(A, B, C, s);
        const bool ok = disc_ok(disc, B) && t >= 0.0 && fabs(fma(t, uz, z)) <= c[22] &&
                        (!SEG || wedge_in_hit(S, fma(t, ux, x), fma(t, uy, y)));
        take(ok, t, 2, best, sid);
    }
    if (SEG) face_entries<kCone>(S, nullptr, x, y, z, ux, uy, uz, best, sid);
    return inside ? 0.0 : best;
}

template <bool SEG>
__device__ __forceinline__ double cone_dist_in(const ShapeRec &S, double x, double y, double z,
                                               double ux, double uy, double uz, int &sid) {
    const double *c = S.c;
    const int hole = S.hole;
    const double dz = c[0];
    const double rsq = x * x + y * y;
    const double wo = fma(c[2], z, c[1]);
    const double wi = fma(c[4], z, c[3]);
    const bool inside = fabs(z) <= dz && rsq <= wo * wo && (!hole || rsq >= wi * wi) &&
                        (!SEG || wedge_in(S, x, y));
    double best = kBig;
    sid = -1;
    take(uz != 0.0, fdiv(dz - (uz > 0.0 ? z : -z), fabs(uz)), 0, best, sid);
    const double A0 = ux * ux + uy * uy;
    const double B0 = x * ux + y * uy;
    {   // leave the outer nappe
        const double v = c[2] * uz;
        const double A = A0 - v * v, B = B0 - v * wo, C = rsq - wo * wo;
        const double disc = B * B - A * C;
        const double s = disc_sqrt(disc, B);
        const double t = root_up(A, B, C, s);
        take(disc_ok(disc, B) && t >= 0.0, t, 1, best, sid);
    }
    if (hole) {  // enter the inner nappe (the hole)
        const double v = c[4] * uz;
        const double A = A0 - v * v, B = B0 - v * wi, C = rsq - wi * wi;
        const double disc = B * B - A * C;
        const double s = disc_sqrt(disc, B);
        const double t = root_down(A, B, C, s);
        take(disc_ok(disc, B) && t >= 0.0, t, 2, best, sid);
    }
    if (SEG) wedge_exit(S, x, y, ux, uy, best, sid);
    return inside ? best : 0.0;
}

// ----------------------------------------------------------------- polycone
// A sequence of connected cone sections (section 3.1). The radii are
// continuous across the planes inside, so those planes bound nothing: the
// surfaces are the two end planes (surface 0) and, per section j, its outer
// nappe (surface 5 + 2 j) and inner nappe (6 + 2 j), each a boundary only for
// z in [z_j, z_{j+1}], which every candidate checks at its hit point. The
// check allows a slack of eps: a line through a kink of the profile (a
// plane between sections) meets the two sections' nappes there, and rounding
// could otherwise put both hit points just outside their ranges. Within eps
// of the plane the two nappes are within |b_j - b_{j+1}| eps of each other.
// Nappe roots on the mirror nappe fall outside the ranges (the radii are
// >= 0 on them). The loops run over the sections, the same for every lane.
__device__ __forceinline__ bool pcon_contains(const PconRec &P, double x, double y, double z) {
    const double rsq = x * x + y * y;
    const int ns = P.nz - 1;
    bool in = false;
    for (int j = 0; j < ns; ++j) {
        const double wo = fma(P.bo[j], z, P.ao[j]);
        const double wi = fma(P.bi[j], z, P.ai[j]);
        const bool hole = (P.hole_mask >> j) & 1;
        in |= z >= P.z[j] && z <= P.z[j + 1] && rsq <= wo * wo && (!hole || rsq >= wi * wi);
    }
    return in;
}

// Membership of a candidate's hit point, with the slack eps on every bound.
__device__ __forceinline__ bool pcon_contains_hit(const PconRec &P, double x, double y, double z) {
    const double rsq = x * x + y * y;
    const int ns = P.nz - 1;
    bool in = false;
    for (int j = 0; j < ns; ++j) {
        const double wo = fma(P.bo[j], z, P.ao[j]) + P.eps;
        const double wi = fmax(fma(P.bi[j], z, P.ai[j]) - P.eps, 0.0);
        in |= z >= P.z[j] - P.eps && z <= P.z[j + 1] + P.eps && rsq <= wo * wo && rsq >= wi * wi;
    }
    return in;
}

// (u, z) in the profile polygon; u is a signed coordinate in a face's plane.
__device__ __forceinline__ bool pcon_in_profile(const PconRec &P, double u, double z) {
    const int ns = P.nz - 1;
    bool in = false;
    for (int j = 0; j < ns; ++j) {
        const double wo = fma(P.bo[j], z, P.ao[j]);
        const double wi = fma(P.bi[j], z, P.ai[j]);
        in |= z >= P.z[j] && z <= P.z[j + 1] && u <= wo && u >= wi;
    }
    return in;
}

template <bool SEG>
__device__ __forceinline__ double pcon_dist_out(const ShapeRec &S, const PconRec &P, double x,
                                                double y, double z, double ux, double uy,
                                                double uz, int &sid) {
    const bool inside = pcon_contains(P, x, y, z) && (!SEG || wedge_in(S, x, y));
    const int ns = P.nz - 1;
    double best = kBig;
    sid = -1;
    {   // bottom plane, from below moving up, landing on its annulus
        const double t = fdiv(P.z[0] - z, uz);
        const double xh = fma(t, ux, x), yh = fma(t, uy, y);
        const double r2 = xh * xh + yh * yh;
        const bool ok = z < P.z[0] && uz > 0.0 && r2 >= P.rin2_0 && r2 <= P.rout2_0 &&
                        (!SEG || wedge_in_hit(S, xh, yh));
        take(ok, t, 0, best, sid);
    }
    {   // top plane, from above moving down
        const double t = fdiv(P.z[ns] - z, uz);
        const double xh = fma(t, ux, x), yh = fma(t, uy, y);
        const double r2 = xh * xh + yh * yh;
        const bool ok = z > P.z[ns] && uz < 0.0 && r2 >= P.rin2_l && r2 <= P.rout2_l &&
                        (!SEG || wedge_in_hit(S, xh, yh));
        take(ok, t, 0, best, sid);
    }
    const double rsq = x * x + y * y;
    const double A0 = ux * ux + uy * uy;
    const double B0 = x * ux + y * uy;
    for (int j = 0; j < ns; ++j) {
        const double zlo = P.z[j] - P.eps, zhi = P.z[j + 1] + P.eps;
        {   // outer nappe: entered where f goes from + to -
            const double w = fma(P.bo[j], z, P.ao[j]);
            const double v = P.bo[j] * uz;
            const double A = A0 - v * v, B = B0 - v * w, C = rsq - w * w;
            const double disc = B * B - A * C;
            const double s = disc_sqrt(disc, B);
            const double t = root_down(A, B, C, s);
            const double zh = fma(t, uz, z);
            const bool ok = disc_ok(disc, B) && t >= 0.0 && zh >= zlo && zh <= zhi &&
                            (!SEG || wedge_in_hit(S, fma(t, ux, x), fma(t, uy, y)));
            take(ok, t, 5 + 2 * j, best, sid);
        }
        if ((P.hole_mask >> j) & 1) {  // inner nappe: left from the hole
            const double w = fma(P.bi[j], z, P.ai[j]);
            const double v = P.bi[j] * uz;
            const double A = A0 - v * v, B = B0 - v * w, C = rsq - w * w;
            const double disc = B * B - A * C;
            const double s = disc_sqrt(disc, B);
            const double t = root_up(A, B, C, s);
            const double zh = fma(t, uz, z);
            const bool ok = disc_ok(disc, B) && t >= 0.0 && zh >= zlo && zh <= zhi &&
                            (!SEG || wedge_in_hit(S, fma(t, ux, x), fma(t, uy, y)));
            take(ok, t, 6 + 2 * j, best, sid);
        }
    }
    if (SEG) face_entries<kPcon>(S, &P, x, y, z, ux, uy, uz, best, sid);
    return inside ? 0.0 : best;
}

template <bool SEG>
__device__ __forceinline__ double pcon_dist_in(const ShapeRec &S, const PconRec &P, double x,
                                               double y, double z, double ux, double uy, double uz,
                                               int &sid) {
    const bool inside = pcon_contains(P, x, y, z) && (!SEG || wedge_in(S, x, y));
    const int ns = P.nz - 1;
    double best = kBig;
    sid = -1;
    take(uz < 0.0, fdiv(P.z[0] - z, uz), 0, best, sid);
    take(uz > 0.0, fdiv(P.z[ns] - z, uz), 0, best, sid);
    const double rsq = x * x + y * y;
    const double A0 = ux * ux + uy * uy;
    const double B0 = x * ux + y * uy;
    for (int j = 0; j < ns; ++j) {
        const double zlo = P.z[j] - P.eps, zhi = P.z[j + 1] + P.eps;
        {   // leave the outer nappe
            const double w = fma(P.bo[j], z, P.ao[j]);
            const double v = P.bo[j] * uz;
            const double A = A0 - v * v, B = B0 - v * w, C = rsq - w * w;
            const double disc = B * B - A * C;
            const double s = disc_sqrt(disc, B);
            const double t = root_up(A, B, C, s);
            const double zh = fma(t, uz, z);
            take(disc_ok(disc, B) && t >= 0.0 && zh >= zlo && zh <= zhi, t, 5 + 2 * j, best, sid);
        }
        if ((P.hole_mask >> j) & 1) {  // enter the hole
            const double w = fma(P.bi[j], z, P.ai[j]);
            const double v = P.bi[j] * uz;
            const double A = A0 - v * v, B = B0 - v * w, C = rsq - w * w;
            const double disc = B * B - A * C;
            const double s = disc_sqrt(disc, B);
            const double t = root_down(A, B, C, s);
            const double zh = fma(t, uz, z);
            take(disc_ok(disc, B) && t >= 0.0 && zh >= zlo && zh <= zhi, t, 6 + 2 * j, best, sid);
        }
    }
    if (SEG) wedge_exit(S, x, y, ux, uy, best, sid);
    return inside ? best : 0.0;
}

// Squared distance from (r, z) to the profile's edges: the two end edges,
// the outer edges and the inner edges; an inner edge on the axis (both radii
// 0) bounds no surface and is skipped unless `axis` is set (a face's
// polygon, whose edge on the axis is real).
__device__ __forceinline__ double pcon_edges_d2(const PconRec &P, double r, double z, bool axis) {
    const int ns = P.nz - 1;
    const double rb = fmin(fmax(r, P.rin[0]), P.rout[0]);
    const double rt = fmin(fmax(r, P.rin[ns]), P.rout[ns]);
    double d2 = fmin(sq(r - rb) + sq(z - P.z[0]), sq(r - rt) + sq(z - P.z[ns]));
    for (int j = 0; j < ns; ++j) {
        const double h = P.z[j + 1] - P.z[j];
        d2 = fmin(d2, seg_d2(r, z, P.rout[j], P.z[j], P.rout[j + 1] - P.rout[j], h, P.inv_eo[j]));
        if (axis || ((P.hole_mask >> j) & 1))
            d2 = fmin(d2, seg_d2(r, z, P.rin[j], P.z[j], P.rin[j + 1] - P.rin[j], h, P.inv_ei[j]));
    }
    return d2;
}

// A solid of revolution: the planar distance from (r, z) to the profile's
// edges, inside and outside alike.
__device__ __forceinline__ double pcon_safety(const PconRec &P, double x, double y, double z) {
    return fsqrt(pcon_edges_d2(P, fsqrt(x * x + y * y), z, false));
}

__device__ __forceinline__ double pcon_face_d2(const PconRec &P, double u, double z) {
    return pcon_in_profile(P, u, z) ? 0.0 : pcon_edges_d2(P, u, z, true);
}

// ------------------------------------------------------ segment safety
// Squared distance from (u, z) to a face, the profile polygon laid in the
// half-plane at phi_i with u along e_i (0 on or inside the polygon). The
// tube's profile is the rectangle [rmin, rmax] x [-dz, dz]; the cone's is the
// trapezoid, its inner edge included even on the axis (there the two faces
// meet).
__device__ __forceinline__ double tube_face_d2(const double *c, double u, double z) {
    const double du = fmax(fmax(c[0] - u, u - c[1]), 0.0);
    const double dz = fmax(fabs(z) - c[2], 0.0);
    return du * du + dz * dz;
}

__device__ __forceinline__ double cone_face_d2(const double *c, double u, double z) {
    const double dz = c[0];
    const double wo = fma(c[2], z, c[1]);
    const double wi = fma(c[4], z, c[3]);
    const bool in = fabs(z) <= dz && u <= wo && u >= wi;
    const double rb = fmin(fmax(u, c[5]), c[6]);
    const double rt = fmin(fmax(u, c[7]), c[8]);
    double d2 = fmin(sq(u - rb) + sq(z + dz), sq(u - rt) + sq(z - dz));
    d2 = fmin(d2, seg_d2(u, z, c[6], -dz, c[8] - c[6], 2.0 * dz, c[15]));
    d2 = fmin(d2, seg_d2(u, z, c[5], -dz, c[7] - c[5], 2.0 * dz, c[16]));
    return in ? 0.0 : d2;
}

// Safety of a segment: the boundary is the base's surfaces within the range
// and the two faces.
//   Outside the solid: the base's Safety if p is in the range (the nearest
//   point of a surface of revolution has p's own azimuth), and the distance
//   to each face, sqrt(v_i^2 + d2_i) with v_i the distance from the face's
//   plane and d2_i that of (u_i, z) to the face polygon (this also covers
//   the base surfaces' edges when p is out of the range).
//   Inside: the base's Safety and, per face, |v_i| when the foot of the
//   perpendicular lies on the face's half-plane (u_i >= 0) or else r. The
//   foot can fall short of the face only into the hole, where the base's
//   inner surface is nearer than |v_i|; off the half-plane the face is at
//   least r away, exactly r where the profile reaches the axis, and with a
//   hole the inner surface is nearer than r.
template <int BASE>
__device__ __forceinline__ double seg_safety(const ShapeRec &S, const PconRec *pc, double x,
                                             double y, double z) {
    const double *c = S.c;
    const double base = BASE == kTube   ? tube_safety(c, S.hole, x, y, z)
                        : BASE == kCone ? cone_safety(c, S.hole, x, y, z)
                                        : pcon_safety(*pc, x, y, z);
    const bool in_base = base_contains<BASE>(S, pc, x, y, z);
    const double a = wedge_a(c, x, y), b = wedge_b(c, x, y);
    const bool in_range = S.convex ? (a >= 0.0 && b >= 0.0) : (a >= 0.0 || b >= 0.0);
    const double u1 = fma(c[18], y, c[17] * x), u2 = fma(c[20], y, c[19] * x);
    const double r = fsqrt(x * x + y * y);
    const double f_in = fmin(u1 >= 0.0 ? fabs(a) : r, u2 >= 0.0 ? fabs(b) : r);
    const double d1 = BASE == kTube   ? tube_face_d2(c, u1, z)
                      : BASE == kCone ? cone_face_d2(c, u1, z)
                                      : pcon_face_d2(*pc, u1, z);
    const double d2 = BASE == kTube   ? tube_face_d2(c, u2, z)
                      : BASE == kCone ? cone_face_d2(c, u2, z)
                                      : pcon_face_d2(*pc, u2, z);
    const double f_out = fsqrt(fmin(fma(a, a, d1), fma(b, b, d2)));
    return (in_base && in_range) ? fmin(base, f_in) : fmin(in_range ? base : kBig, f_out);
}

// ------------------------------------------------------ dispatch on kind
// `pc` is the shape's polycone record (read only for the polycone kinds).
template <int KIND>
__device__ __forceinline__ bool shape_contains(const ShapeRec &s, const PconRec *pc, double x,
                                               double y, double z) {
    if (KIND == kBox) return box_contains(s.c, x, y, z);
    if (KIND == kTube) return tube_contains(s.c, x, y, z);
    if (KIND == kCone) return cone_contains(s.c, s.hole, x, y, z);
    if (KIND == kTubs) return tube_contains(s.c, x, y, z) && wedge_in(s, x, y);
    if (KIND == kCons) return cone_contains(s.c, s.hole, x, y, z) && wedge_in(s, x, y);
    if (KIND == kPcon) return pcon_contains(*pc, x, y, z);
    return pcon_contains(*pc, x, y, z) && wedge_in(s, x, y);
}

template <int KIND>
__device__ __forceinline__ double shape_safety(const ShapeRec &s, const PconRec *pc, double x,
                                               double y, double z) {
    if (KIND == kBox) return box_safety(s.c, x, y, z);
    if (KIND == kTube) return tube_safety(s.c, s.hole, x, y, z);
    if (KIND == kCone) return cone_safety(s.c, s.hole, x, y, z);
    if (KIND == kTubs) return seg_safety<kTube>(s, pc, x, y, z);
    if (KIND == kCons) return seg_safety<kCone>(s, pc, x, y, z);
    if (KIND == kPcon) return pcon_safety(*pc, x, y, z);
    return seg_safety<kPcon>(s, pc, x, y, z);
}

template <int KIND>
__device__ __forceinline__ double shape_dist_out(const ShapeRec &s, const PconRec *pc, double x,
                                                 double y, double z, double ux, double uy,
                                                 double uz, int &sid) {
    if (KIND == kBox) return box_dist_out(s.c, x, y, z, ux, uy, uz, sid);
    if (KIND == kTube) return tube_dist_out<false>(s, x, y, z, ux, uy, uz, sid);
    if (KIND == kCone) return cone_dist_out<false>(s, x, y, z, ux, uy, uz, sid);
    if (KIND == kTubs) return tube_dist_out<true>(s, x, y, z, ux, uy, uz, sid);
    if (KIND == kCons) return cone_dist_out<true>(s, x, y, z, ux, uy, uz, sid);
    if (KIND == kPcon) return pcon_dist_out<false>(s, *pc, x, y, z, ux, uy, uz, sid);
    return pcon_dist_out<true>(s, *pc, x, y, z, ux, uy, uz, sid);
}

template <int KIND>
__device__ __forceinline__ double shape_dist_in(const ShapeRec &s, const PconRec *pc, double x,
                                                double y, double z, double ux, double uy,
                                                double uz, int &sid) {
    if (KIND == kBox) return box_dist_in(s.c, x, y, z, ux, uy, uz, sid);
    if (KIND == kTube) return tube_dist_in<false>(s, x, y, z, ux, uy, uz, sid);
    if (KIND == kCone) return cone_dist_in<false>(s, x, y, z, ux, uy, uz, sid);
    if (KIND == kTubs) return tube_dist_in<true>(s, x, y, z, ux, uy, uz, sid);
    if (KIND == kCons) return cone_dist_in<true>(s, x, y, z, ux, uy, uz, sid);
    if (KIND == kPcon) return pcon_dist_in<false>(s, *pc, x, y, z, ux, uy, uz, sid);
    return pcon_dist_in<true>(s, *pc, x, y, z, ux, uy, uz, sid);
}

// `kind` is uniform across the wavefront wherever these are called. KSET
// bounds the kinds a geometry holds (kSetBasic: box, tube, cone; kSetSeg:
// and their segments; kSetAll: and polycones), so that kernels for simpler
// geometries carry no code for the kinds they never meet: the navigator's
// loop body stays small, which the instruction cache rewards.
enum : int { kSetBasic = 0, kSetSeg = 1, kSetAll = 2 };

#define GN_KIND_SWITCH(CALL) GN_KIND_SWITCH_ON(s.kind, CALL)
#define GN_KIND_SWITCH_ON(KIND, CALL)       \
    if (KSET == kSetBasic) {                \
        switch (KIND) {                     \
            case kBox: return CALL(kBox);   \
            case kTube: return CALL(kTube); \
            default: return CALL(kCone);    \
        }                                   \
    }                                       \
    if (KSET == kSetSeg) {                  \
        switch (KIND) {                     \
            case kBox: return CALL(kBox);   \
            case kTube: return CALL(kTube); \
            case kCone: return CALL(kCone); \
            case kTubs: return CALL(kTubs); \
            default: return CALL(kCons);    \
        }                                   \
    }                                       \
    switch (KIND) {                         \
        case kBox: return CALL(kBox);       \
        case kTube: return CALL(kTube);     \
        case kCone: return CALL(kCone);     \
        case kTubs: return CALL(kTubs);     \
        case kCons: return CALL(kCons);     \
        case kPcon: return CALL(kPcon);     \
        default: return CALL(kPcons);       \
    }

template <int KSET = kSetAll>
__device__ __forceinline__ bool any_contains(const ShapeRec &s, const PconRec *pc, double x,
                                             double y, double z) {
#define GN_CALL(K) shape_contains<K>(s, pc, x, y, z)
    GN_KIND_SWITCH(GN_CALL)
#undef GN_CALL
}

template <int KSET = kSetAll>
__device__ __forceinline__ double any_safety(const ShapeRec &s, const PconRec *pc, double x,
                                             double y, double z) {
#define GN_CALL(K) shape_safety<K>(s, pc, x, y, z)
    GN_KIND_SWITCH(GN_CALL)
#undef GN_CALL
}

template <int KSET = kSetAll>
__device__ __forceinline__ double any_dist_out(const ShapeRec &s, const PconRec *pc, double x,
                                               double y, double z, double ux, double uy,
                                               double uz, int &sid) {
#define GN_CALL(K) shape_dist_out<K>(s, pc, x, y, z, ux, uy, uz, sid)
    GN_KIND_SWITCH(GN_CALL)
#undef GN_CALL
}

template <int KSET = kSetAll>
__device__ __forceinline__ double any_dist_in(const ShapeRec &s, const PconRec *pc, double x,
                                              double y, double z, double ux, double uy,
                                              double uz, int &sid) {
#define GN_CALL(K) shape_dist_in<K>(s, pc, x, y, z, ux, uy, uz, sid)
    GN_KIND_SWITCH(GN_CALL)
#undef GN_CALL
}

// Number of kind classes a kind set tells apart (kinds beyond them take the
// last class's code, as in the switch above), and the class of a kind.
template <int KSET>
__device__ __forceinline__ constexpr int kind_classes() {
    return KSET == kSetBasic ? 3 : (KSET == kSetSeg ? 5 : 7);
}
template <int KSET>
__device__ __forceinline__ int kind_class(int kind) {
    return kind < kind_classes<KSET>() - 1 ? kind : kind_classes<KSET>() - 1;
}

// DistFromOutside for a class known to be uniform over the wavefront (a
// scalar branch instead of one path per kind present).
template <int KSET>
__device__ __forceinline__ double class_dist_out(int cls, const ShapeRec &s, const PconRec *pc, double x,
                                                 double y, double z, double ux, double uy, double uz,
                                                 int &sid) {
#define GN_CALL(K) shape_dist_out<K>(s, pc, x, y, z, ux, uy, uz, sid)
    GN_KIND_SWITCH_ON(cls, GN_CALL)
#undef GN_CALL
}
#undef GN_KIND_SWITCH
#undef GN_KIND_SWITCH_ON

// The mother's DistFromInside for the navigators; SURF false: the surface
// that sets it is not wanted (sid = -1), and a box mother takes box_exit.
template <bool SURF, int KSET>
__device__ __forceinline__ double mother_step(const VolumeRec &v, double x, double y, double z, double ux,
                                              double uy, double uz, int &sid) {
    if (!SURF && v.mother.kind == kBox) {
        sid = -1;
        return box_exit(v.mother.c, x, y, z, ux, uy, uz);
    }
    return any_dist_in<KSET>(v.mother, v.pcon, x, y, z, ux, uy, uz, sid);
}

// Outward-or-inward normal (any scale/sign) of surface `sid` at local point h.
__device__ __forceinline__ void surface_normal(const ShapeRec &s, const PconRec *pc, int sid,
                                               double hx, double hy, double hz, double &nx,
                                               double &ny, double &nz) {
    nx = ny = nz = 0.0;
    if (s.kind == kBox) {
        nx = sid == 0 ? 1.0 : 0.0;
        ny = sid == 1 ? 1.0 : 0.0;
        nz = sid == 2 ? 1.0 : 0.0;
        return;
    }
    if (sid == 0) { nz = 1.0; return; }
    if (sid < 0) return;
    if (sid == 3) {  // segment face planes: n1, n2
        nx = -s.c[18];
        ny = s.c[17];
        return;
    }
    if (sid == 4) {
        nx = s.c[20];
        ny = -s.c[19];
        return;
    }
    nx = hx;
    ny = hy;
    if (s.kind == kPcon || s.kind == kPcons) {  // nappe of section j: r = a + b z
        const int j = (sid - 5) >> 1;
        const bool outer = ((sid - 5) & 1) == 0;
        const double a = outer ? pc->ao[j] : pc->ai[j];
        const double b = outer ? pc->bo[j] : pc->bi[j];
        nz = -b * fma(b, hz, a);
        return;
    }
    if (s.kind == kCone || s.kind == kCons) {
        const double a = sid == 1 ? s.c[1] : s.c[3];
        const double b = sid == 1 ? s.c[2] : s.c[4];
        nz = -b * fma(b, hz, a);
    }
}

// ----------------------------------------------------------- navigator
// Per-track navigator of Fig. 1b, sequential form (the adjoint's forward
// recomputation, and the forward navigators with culling off): the mother's
// DistFromInside, then each daughter's DistFromOutside in its own frame,
// keeping the smallest (ties to the mother, then the lowest index).
// Daughters are walked in lockstep by the whole wavefront, so the daughter
// record and its kind are uniform (scalar loads, scalar branch).
//
// With COUNT, the work done is tallied into census[kCensusSlots] (one atomic
// per wavefront and event, adding the number of active lanes): slots
// 2 * kind + hole count daughter evaluations, slot kCensusCull culling
// tests, slot kCensusTracks tracks.
__device__ __forceinline__ void census_add(unsigned long long *census, int slot) {
    const unsigned long long act = __ballot(1);
    if ((int)__lane_id() == __ffsll((unsigned long long)act) - 1)
        atomicAdd(&census[slot], (unsigned long long)__popcll(act));
}

template <bool HAS_OFFS, bool TRACK_SURF, bool COUNT = false, int KSET = kSetAll>
__device__ __forceinline__ void nav_track(const VolumeRec &v, const DaughterRec *__restrict__ dau,
                                          const CullRec *__restrict__ cul,
                                          const double *__restrict__ offs, double x, double y,
                                          double z, double ux, double uy, double uz, double &best,
                                          int &hit, int &bsid,
                                          unsigned long long *census = nullptr) {
    int sid;
    if (COUNT) census_add(census, kCensusTracks);
    best = mother_step<TRACK_SURF, KSET>(v, x, y, z, ux, uy, uz, sid);
    hit = -1;
    bsid = sid;
    const int nd = v.nd;
    for (int k = 0; k < nd; ++k) {
        const CullRec &Q = cul[k];
        double wx = x - Q.tx, wy = y - Q.ty, wz = z - Q.tz;
        if (HAS_OFFS) {
            wx -= offs[3 * k + 0];
            wy -= offs[3 * k + 1];
            wz -= offs[3 * k + 2];
        }
        const DaughterRec &D = dau[k];
        if (COUNT) census_add(census, 2 * D.shape.kind + D.shape.hole);
        const double *R = D.rot;
        // local = R^T w
        const double lx = fma(R[6], wz, fma(R[3], wy, R[0] * wx));
        const double ly = fma(R[7], wz, fma(R[4], wy, R[1] * wx));
        const double lz = fma(R[8], wz, fma(R[5], wy, R[2] * wx));
        const double lux = fma(R[6], uz, fma(R[3], uy, R[0] * ux));
        const double luy = fma(R[7], uz, fma(R[4], uy, R[1] * ux));
        const double luz = fma(R[8], uz, fma(R[5], uy, R[2] * ux));
        const double s = any_dist_out<KSET>(D.shape, D.pcon, lx, ly, lz, lux, luy, luz, sid);
        const bool better = s < best;
        best = better ? s : best;
        hit = better ? k : hit;
        if (TRACK_SURF) bsid = better ? sid : bsid;
    }
    best = best == 0.0 ? 0.0 : best;  // a step of -0 is reported as +0
}

// ------------------------------------------------ compacted navigator
// Culling: a (track, daughter) pair needs evaluating only when the track's
// half-line from p passes within the daughter's culling radius (its
// bounding radius enlarged by 1e-6 relative + 1e-6) of the sphere's centre
// T; otherwise the daughter cannot be entered at any t >= 0, so it could
// neither lower the step nor win a tie. (The mother's exit would bound the
// half-line further, but the daughters lie inside the mother and no line
// comes back near them after leaving a convex mother: on the batched
// workload that bound removes no pair, and leaving it out saves a min per
// test.) Skipping a daughter for a whole wavefront unless some lane needs
// it would leave all 64 lanes evaluating it for the one lane or two that do
// (with random tracks about one lane in 64). The compacted form separates the
// two: the wavefront first runs the culling tests of its tracks against
// every daughter (lockstep: the culling record is uniform) and appends each
// (track, daughter) pair that passes to a queue in LDS; then each lane takes
// one queued pair and evaluates that daughter's DistFromOutside for that
// track, so a batch of 64 pairs costs one pass (the lanes of different kinds
// take their kinds' code in turn).
//
// The step of a track is the minimum over its candidates of (s, index),
// compared lexicographically with the mother as index -1: the result of
// the sequential loop, whose strict < keeps the earlier of equal steps.
// Each track's running minimum sits in LDS as a 64-bit key (an
// order-preserving map of the double, -0 taken as +0, so that a step of -0
// is reported as +0 as in the sequential loop) and an index (packed with the
// surface that set the step, see hit_pack); a batch merges into it with a
// 64-bit LDS min on the key, then, for the pairs whose key equals the new
// minimum, an integer min on the index (reset first when the batch lowered
// the key). After every batch the slot holds the lexicographic minimum of
// all candidates merged so far, whatever the order of the batches.
//
// At the end of its round, each track that queued a pair takes a slot of
// the wavefront's track cache in LDS, which holds its six coordinates; the
// batches read their tracks from there rather than from global memory,
// where the six component arrays put each track on six cache lines, long
// evicted from L2 by the time its batch runs. (Pairs flushed within their
// own round, when the queue fills or the slots run out, read their track
// from global memory while it is still cached.) A flush empties the queue
// and the slots. The queue is flushed when a chunk's pairs could overflow
// it, when a round's tracks would overflow the slots, and at the end of the
// tile.
//
// Queue entries pack the daughter index (bits 10..31) and the track's index
// within the tile, round * 64 + lane (bits 0..9). All LDS traffic of the
// queue, the slots and the minima is the wavefront's own, whose LDS
// instructions execute in program order, so no barrier is needed.
constexpr int kQueueCap = 512;
constexpr int kPoolMax = 128;
constexpr int kSlots = 48;
constexpr unsigned char kNoSlot = 255;
template <int U>
struct NavScratch {
    unsigned long long key[U * 64];   // running minimum per track: key of the step
    int hit[U * 64];                  // and the packed index of its candidate
    unsigned char slot_of[U * 64];    // the track's slot, kNoSlot if none
    double x[kSlots], y[kSlots], z[kSlots], ux[kSlots], uy[kSlots], uz[kSlots];
    union {
        unsigned int queue[kQueueCap];  // (daughter << 10) | round * 64 + lane
        struct {                        // a pooled flush of at most kPoolMax pairs:
            unsigned int entry[kPoolMax];          // the queue's entries
            unsigned long long key[kPoolMax];      // each pair's step key
            int hit[kPoolMax];                     // and packed hit
        } pooled;
    };
    static_assert(U * 64 <= 1024, "track index within the tile: 10 bits");
    static_assert(sizeof(pooled) <= sizeof(queue), "pooled results within the queue");
};
static_assert(kSlots < kNoSlot, "slot numbers");

// Scratch of the compacted safety and localization (one round of 64 points
// per wavefront): running minima per point and the queue of (point,
// daughter) pairs, (daughter << 10) | point.
struct PointQueue {
    unsigned long long key[64];
    int hit[64];
    unsigned int queue[kQueueCap];
};

// A NaN daughter step never wins and a NaN mother step is never beaten, as
// in the sequential loop.
__device__ __forceinline__ unsigned long long step_key(double s, bool mother = false) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(s == 0.0 ? 0.0 : s);
    const unsigned long long k = (b >> 63) ? ~b : (b | 0x8000000000000000ull);
    return s == s ? k : (mother ? 0ull : ~0ull);
}
__device__ __forceinline__ double key_step(unsigned long long k) {
    return __longlong_as_double((long long)((k >> 63) ? (k & 0x7fffffffffffffffull) : ~k));
}

// Accesses to the running minima, which other lanes of the wavefront update
// atomically, and to the slots, which other lanes read.
template <typename T>
__device__ __forceinline__ T lds_load(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}
template <typename T>
__device__ __forceinline__ void lds_store(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// Number of set bits of m below this lane.
__device__ __forceinline__ int lanes_below(unsigned long long m) {
    return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                          __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

// DistFromOutside of daughter k (records D, Q) for a mother-frame track;
// sid receives the surface that set it. With a class cls >= 0 (uniform over
// the wavefront), the daughter is known to be of that kind class.
template <bool HAS_OFFS, int KSET>
__device__ __forceinline__ double daughter_dist_out(const DaughterRec &D, const CullRec &Q,
                                                    const double *__restrict__ offs, int k, double x,
                                                    double y, double z, double ux, double uy,
                                                    double uz, int &sid, int cls = -1) {
    double wx = x - Q.tx, wy = y - Q.ty, wz = z - Q.tz;
    if (HAS_OFFS) {
        wx -= offs[3 * k + 0];
        wy -= offs[3 * k + 1];
        wz -= offs[3 * k + 2];
    }
    const double *R = D.rot;
    const double lx = fma(R[6], wz, fma(R[3], wy, R[0] * wx));
    const double ly = fma(R[7], wz, fma(R[4], wy, R[1] * wx));
    const double lz = fma(R[8], wz, fma(R[5], wy, R[2] * wx));
    const double lux = fma(R[6], uz, fma(R[3], uy, R[0] * ux));
    const double luy = fma(R[7], uz, fma(R[4], uy, R[1] * ux));
    const double luz = fma(R[8], uz, fma(R[5], uy, R[2] * ux));
    if (cls >= 0) return class_dist_out<KSET>(cls, D.shape, D.pcon, lx, ly, lz, lux, luy, luz, sid);
    return any_dist_out<KSET>(D.shape, D.pcon, lx, ly, lz, lux, luy, luz, sid);
}

// A tile's six track arrays from its first track on: uniform pointers, so
// that a lane's track, an unsigned index below 1024 off them, is loaded with
// a scalar base address and a 32-bit vector offset (no 64-bit address per
// lane and array).
struct TileTracks {
    const double *x, *y, *z, *ux, *uy, *uz;
};
// element j (< 2^29) of a, its byte offset formed in 32 bits
template <typename T>
__device__ __forceinline__ T &at32(T *a, unsigned int j) {
    return *reinterpret_cast<T *>(reinterpret_cast<char *>(a) + j * (unsigned int)sizeof(T));
}
template <typename T>
__device__ __forceinline__ const T &at32(const T *a, unsigned int j) {
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(a) + j * (unsigned int)sizeof(T));
}
__device__ __forceinline__ TileTracks tile_tracks(const TracksDev &t, int64_t base) {
    TileTracks r;
    r.x = t.x + base;
    r.y = t.y + base;
    r.z = t.z + base;
    r.ux = t.ux + base;
    r.uy = t.uy + base;
    r.uz = t.uz + base;
    return r;
}

// A hit slot holds the candidate's index k (-1 for the mother) and the
// surface that set its step (sid, -1 .. 254) as k * 256 + sid + 1: ordered
// by k, since each index has one candidate per track, and the adjoint reads
// the winner's surface back without evaluating it again.
__device__ __forceinline__ int hit_pack(int k, int sid) { return k * 256 + (sid + 1); }
__device__ __forceinline__ int hit_index(int v) { return v >> 8; }
__device__ __forceinline__ int hit_surface(int v) { return (v & 255) - 1; }

// Merges a candidate (its step's key and packed hit) into running minimum j
// of S, the wavefront's own. Lanes of one call may share a minimum; whatever
// the order of calls, it ends at the lexicographic minimum of all candidates
// merged. merge_step: the same for candidate (s, k) with surface sid.
template <typename Scratch>
__device__ __forceinline__ void merge_key(Scratch &S, int j, unsigned long long key, int hp) {
    const unsigned long long before = lds_load(&S.key[j]);
    __hip_atomic_fetch_min(&S.key[j], key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    const unsigned long long now = lds_load(&S.key[j]);
    if (now < before) lds_store(&S.hit[j], 0x7fffffff);
    if (key == now) __hip_atomic_fetch_min(&S.hit[j], hp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}
template <typename Scratch>
__device__ __forceinline__ void merge_step(Scratch &S, int j, double s, int k, int sid) {
    merge_key(S, j, step_key(s), hit_pack(k, sid));
}

// Runs the qn queued pairs in batches of 64 (one pair per lane), each
// reading its track from its slot, or from global memory if the track has
// none (pairs flushed within their own round), then empties the queue and
// the slots.
template <int U, bool HAS_OFFS, bool COUNT, int KSET, bool SURF>
__device__ __forceinline__ void nav_flush(const DaughterRec *__restrict__ dau,
                                          const CullRec *__restrict__ cul,
                                          const double *__restrict__ offs, const TracksDev &t,
                                          int64_t base, NavScratch<U> &S, int &qn, int &ns, int lane,
                                          unsigned long long *census) {
    for (int e0 = 0; e0 < qn; e0 += 64) {
        const int e = e0 + lane;
        const bool on = e < qn;
        const unsigned int q = on ? S.queue[e] : 0u;
        const int j = (int)(q & 1023u);
        const int k = (int)(q >> 10);
        if (COUNT) {
            const int c = 2 * dau[k].shape.kind + dau[k].shape.hole;
            for (int cc = 0; cc < 2 * (kPcons + 1); ++cc) {
                const unsigned long long m = __ballot(on && c == cc);
                if (m != 0ull && lane == __ffsll(m) - 1) atomicAdd(&census[cc], (unsigned long long)__popcll(m));
            }
        }
        if (on) {
            const int sl = lds_load(&S.slot_of[j]);
            double x, y, z, ux, uy, uz;
            if (sl != kNoSlot) {
                x = lds_load(&S.x[sl]);
                y = lds_load(&S.y[sl]);
                z = lds_load(&S.z[sl]);
                ux = lds_load(&S.ux[sl]);
                uy = lds_load(&S.uy[sl]);
                uz = lds_load(&S.uz[sl]);
            } else {
                const TileTracks tt = tile_tracks(t, base);
                const unsigned int ju = (unsigned int)j;
                x = at32(tt.x, ju);
                y = at32(tt.y, ju);
                z = at32(tt.z, ju);
                ux = at32(tt.ux, ju);
                uy = at32(tt.uy, ju);
                uz = at32(tt.uz, ju);
            }
            int sid;
            const double s = daughter_dist_out<HAS_OFFS, KSET>(dau[k], cul[k], offs, k, x, y, z, ux, uy, uz, sid);
            merge_step(S, j, s, k, SURF ? sid : -1);  // (a surface not wanted is not tracked)
        }
    }
    qn = 0;
    ns = 0;
}

// Per-track constants of the culling test: the unit direction e (as -e),
// and for the expanded form (no offsets) |p|^2, p.e, -2 p; a zero
// direction, or one whose |d|^2 overflows, gives e = 0 (the test then
// takes the start point).
__device__ __forceinline__ void cull_constants(double x, double y, double z, double ux, double uy, double uz,
                                               double &pp, double &pe, double &mpx, double &mpy, double &mpz,
                                               double &mex, double &mey, double &mez) {
    const double dd = fma(uz, uz, fma(uy, uy, ux * ux));
    const double il = (dd > 0.0 && dd < __builtin_inf()) ? rsqrt_fine(dd) : 0.0;
    pp = fma(z, z, fma(y, y, x * x));
    pe = fma(z, uz, fma(y, uy, x * ux)) * il;
    mpx = -2.0 * x;
    mpy = -2.0 * y;
    mpz = -2.0 * z;
    mex = -ux * il;
    mey = -uy * il;
    mez = -uz * il;
}

// Navigates the tracks base + u * 64 + lane (u < U, index below `count`
// past base) of one volume, leaving each track's step (as a key) and hit
// index in S; with SURF, the hit slot also carries the surface that set the
// step (for the adjoint).
//
// Without FINAL the last flush is left to the caller: the queue's length is
// returned, its tracks holding slots.
//
// With SHIFTED (offsets only), the culling tests take their records from
// `shifted`: the centres moved by this call's offsets and the thresholds of
// the expanded test for them (k_shift_cull), so that they run as without
// offsets; the queued pairs still form w = p - T - offset from the
// unshifted records, as every other form does.
template <int U, bool HAS_OFFS, bool COUNT, int KSET, bool SURF = true, bool FINAL = true, bool SHIFTED = false>
__device__ __forceinline__ int nav_compact_core(const VolumeRec &v, const DaughterRec *__restrict__ dau,
                                                const CullRec *__restrict__ cul,
                                                const double *__restrict__ offs, const TracksDev &t,
                                                int64_t base, int count, NavScratch<U> &S, int lane,
                                                unsigned long long *census = nullptr,
                                                const CullRec *__restrict__ shifted = nullptr) {
    static_assert(!SHIFTED || HAS_OFFS, "shifted culling records go with offsets");
    constexpr bool EXPLICIT = HAS_OFFS && !SHIFTED;  // tests that form w = p - T - offset
    const CullRec *__restrict__ tcul = SHIFTED ? shifted : cul;
    int qn = 0;  // queue length (uniform)
    int ns = 0;  // slots in use (uniform)
    const int nd = v.nd;
    const int ndp = (nd + kCullChunk - 1) / kCullChunk * kCullChunk;
#pragma unroll 1
    for (int u = 0; u < U; ++u) {
        if (u * 64 >= count) break;
        const int j = u * 64 + lane;
        const bool act = j < count;
        const unsigned long long amask = __builtin_amdgcn_ballot_w64(act);
        const TileTracks tt = tile_tracks(t, base);
        const unsigned int ju = act ? (unsigned int)j : 0u;
        double x = at32(tt.x, ju), y = at32(tt.y, ju), z = at32(tt.z, ju);
        double ux = at32(tt.ux, ju), uy = at32(tt.uy, ju), uz = at32(tt.uz, ju);
        if (COUNT && lane == 0) atomicAdd(&census[kCensusTracks], (unsigned long long)__popcll(amask));
        int sid;
        const double ms = mother_step<SURF, KSET>(v, x, y, z, ux, uy, uz, sid);
        lds_store(&S.key[j], step_key(ms, true));
        lds_store(&S.hit[j], hit_pack(-1, sid));
        lds_store(&S.slot_of[j], kNoSlot);
        unsigned long long pend = 0ull;  // lanes whose track has queued pairs (uniform)
        double pp, pe, mpx, mpy, mpz, mex, mey, mez;
        cull_constants(x, y, z, ux, uy, uz, pp, pe, mpx, mpy, mpz, mex, mey, mez);
        // a lane past the tile's end gets |p|^2 = +inf: its expanded tests
        // never pass, so their ballots need no mask
        if (!act) pp = __builtin_inf();
        // Daughters in chunks of kCullChunk (the tables are padded to whole
        // chunks with records that never pass): the tests of a chunk run
        // back to back, then its pairs are appended (after a flush if they
        // would overflow the queue or their tracks the slots).
        for (int k0 = 0; k0 < ndp; k0 += kCullChunk) {
            // the chunk's records, loaded together (scalar loads), with
            // their offsets (padding records take daughter 0's: they never
            // pass)
            double ctx[kCullChunk], cty[kCullChunk], ctz[kCullChunk], clim[kCullChunk];
            double cox[kCullChunk], coy[kCullChunk], coz[kCullChunk];
#pragma unroll
            for (int kk = 0; kk < kCullChunk; ++kk) {
                const CullRec &Q = tcul[k0 + kk];
                ctx[kk] = Q.tx;
                cty[kk] = Q.ty;
                ctz[kk] = Q.tz;
                clim[kk] = EXPLICIT ? dau[k0 + kk].cull_r2 : Q.q;
                if (EXPLICIT) {
                    const int ko = k0 + kk < nd ? k0 + kk : 0;
                    cox[kk] = offs[3 * ko + 0];
                    coy[kk] = offs[3 * ko + 1];
                    coz[kk] = offs[3 * ko + 2];
                }
            }
            // the chunk's tests (independent, so they interleave)
            unsigned long long cm[kCullChunk];
#pragma unroll
            for (int kk = 0; kk < kCullChunk; ++kk) {
                double b, g;  // w.e and |w|^2 - shift, with w = p - centre
                if (EXPLICIT) {
                    // the centre moves with the offset: w formed explicitly, shift 0,
                    // limit r2
                    const double wx = x - ctx[kk] - cox[kk];
                    const double wy = y - cty[kk] - coy[kk];
                    const double wz = z - ctz[kk] - coz[kk];
                    b = fma(wz, -mez, fma(wy, -mey, wx * -mex));
                    g = fma(wz, wz, fma(wy, wy, wx * wx));
                } else {
                    // shift |T|^2, limit q (its rounding bound included)
                    b = fma(ctz[kk], mez, fma(cty[kk], mey, fma(ctx[kk], mex, pe)));
                    g = fma(ctz[kk], mpz, fma(cty[kk], mpy, fma(ctx[kk], mpx, pp)));
                }
                const double lim = clim[kk];
                // squared distance from T to the half-line, less the shift:
                // |w|^2 - (w.e)^2 when the line's nearest point lies ahead
                // (w.e < 0), else |w|^2
                const double bn = fmin(b, 0.0);
                const double f = fma(-bn, bn, g);
                // lanes past the tile's end are masked out (the expanded form
                // excludes them through |p|^2)
                const unsigned long long pass = __builtin_amdgcn_ballot_w64(f <= lim);
                cm[kk] = EXPLICIT ? (pass & amask) : pass;
            }
            if (COUNT && lane == 0)
                atomicAdd(&census[kCensusCull],
                          (unsigned long long)__popcll(amask) * (unsigned long long)min(kCullChunk, nd - k0));
            const unsigned long long any = (cm[0] | cm[1]) | (cm[2] | cm[3]);
            static_assert(kCullChunk == 4, "chunk epilogue");
            if (any == 0ull) continue;
            if (qn > kQueueCap - 64 * kCullChunk) {  // the chunk's pairs could overflow the queue
                nav_flush<U, HAS_OFFS, COUNT, KSET, SURF>(dau, cul, offs, t, base, S, qn, ns, lane, census);
                pend = 0ull;
                // the track and its test constants are read and formed again
                // rather than kept live through the flush's evaluations
                x = at32(tt.x, ju);
                y = at32(tt.y, ju);
                z = at32(tt.z, ju);
                ux = at32(tt.ux, ju);
                uy = at32(tt.uy, ju);
                uz = at32(tt.uz, ju);
                cull_constants(x, y, z, ux, uy, uz, pp, pe, mpx, mpy, mpz, mex, mey, mez);
                if (!act) pp = __builtin_inf();
            }
            pend |= any;
#pragma unroll
            for (int kk = 0; kk < kCullChunk; ++kk) {
                const unsigned long long m = cm[kk];
                if (__builtin_amdgcn_inverse_ballot_w64(m))
                    S.queue[qn + lanes_below(m)] = ((unsigned int)(k0 + kk) << 10) | (unsigned int)j;
                qn += __popcll(m);
            }
        }
        // the round's tracks with queued pairs take slots (after a flush if
        // there are too few: the pairs then read their tracks from global
        // memory while they are still in the cache)
        if (pend != 0ull) {
            if (ns + __popcll(pend) > kSlots) {
                nav_flush<U, HAS_OFFS, COUNT, KSET, SURF>(dau, cul, offs, t, base, S, qn, ns, lane, census);
            } else {
                if (__builtin_amdgcn_inverse_ballot_w64(pend)) {
                    const int sl = ns + lanes_below(pend);
                    lds_store(&S.x[sl], x);
                    lds_store(&S.y[sl], y);
                    lds_store(&S.z[sl], z);
                    lds_store(&S.ux[sl], ux);
                    lds_store(&S.uy[sl], uy);
                    lds_store(&S.uz[sl], uz);
                    lds_store(&S.slot_of[j], (unsigned char)sl);
                }
                ns += __popcll(pend);
            }
        }
    }
    if (FINAL) nav_flush<U, HAS_OFFS, COUNT, KSET, SURF>(dau, cul, offs, t, base, S, qn, ns, lane, census);
    return qn;
}

// Writes step, hit and (when HITPT) the hit point of the tile's tracks
// from their running minima.
template <int U, bool HITPT>
__device__ __forceinline__ void nav_write(const NavScratch<U> &S, const TracksDev &t, int64_t base,
                                          int count, int lane, double *__restrict__ step,
                                          int32_t *__restrict__ hit, double *__restrict__ hitpt) {
#pragma unroll 1
    for (int u = 0; u < U; ++u) {
        const int j = u * 64 + lane;
        if (j < count) {
            const unsigned int ju = (unsigned int)j;
            const double s = key_step(lds_load(&S.key[j]));
            at32(step + base, ju) = s;
            at32(hit + base, ju) = hit_index(lds_load(&S.hit[j]));
            if (HITPT) {
                const int64_t n = t.n;
                const TileTracks tt = tile_tracks(t, base);
                at32(hitpt + base, ju) = fma(s, at32(tt.ux, ju), at32(tt.x, ju));
                at32(hitpt + n + base, ju) = fma(s, at32(tt.uy, ju), at32(tt.y, ju));
                at32(hitpt + 2 * n + base, ju) = fma(s, at32(tt.uz, ju), at32(tt.z, ju));
            }
        }
    }
}

// The navigator of one wavefront's tile, writing its outputs.
template <int U, bool HAS_OFFS, bool HITPT, bool COUNT, int KSET>
__device__ __forceinline__ void nav_compact(const VolumeRec &v, const DaughterRec *__restrict__ dau,
                                            const CullRec *__restrict__ cul,
                                            const double *__restrict__ offs, const TracksDev &t,
                                            int64_t base, int count, NavScratch<U> &S, int lane,
                                            double *__restrict__ step, int32_t *__restrict__ hit,
                                            double *__restrict__ hitpt,
                                            unsigned long long *census = nullptr) {
    nav_compact_core<U, HAS_OFFS, COUNT, KSET, false>(v, dau, cul, offs, t, base, count, S, lane, census);
    nav_write<U, HITPT>(S, t, base, count, lane, step, hit, hitpt);
}

// --------------------------------------------- workgroup-pooled last flush
// A tile's last flush holds a few dozen pairs (about 0.12 per track on the
// toy detectors), one batch whose lanes meet every daughter kind the volume
// holds, so that batch runs each kind's code in turn, each on a few lanes.
// Instead, the W wavefronts of a workgroup pool their last queues: each
// sorts its own queue by kind class; after a barrier the workgroup's pairs
// of each class are cut into batches of 64, and the batches, in class order,
// are dealt to the wavefronts in turn, so that each batch runs one class's
// code. A pair's result (key and packed hit) goes back to its place in the
// owner's queue; after a second barrier each wavefront merges its own
// queue's results into its running minima, as a flush of its own would.
// Without `shared` (uniform over the workgroup: its wavefronts' work is too
// uneven to wait for each other) each wavefront flushes its own queue
// alone, with no barrier. (Sorting a single wavefront's queue by class
// saves nothing: its classes still run one after another.)
constexpr int kClassSlots = 8;
template <int W>
struct PoolInfo {
    int cnt[W][kClassSlots];  // pairs of each kind class in each wavefront's sorted queue
    int64_t base[W];          // the wavefront's first track
    int first[W];             // its volume's first daughter and culling record
};

template <int U, int W, bool HAS_OFFS, int KSET, bool SURF>
__device__ __forceinline__ void pool_flush(const DaughterRec *__restrict__ dau_all,
                                           const CullRec *__restrict__ cul_all,
                                           const double *__restrict__ offs, const TracksDev &t,
                                           NavScratch<U> *scr, PoolInfo<W> &P, bool shared, int wave,
                                           int first, int64_t base, int qn, int lane) {
    constexpr int NK = kind_classes<KSET>();
    static_assert(NK <= kClassSlots, "class slots");
    static_assert(kPoolMax == 128, "two entries per lane");
    wave = __builtin_amdgcn_readfirstlane(wave);  // (uniform: the batch loop runs on scalars)
    NavScratch<U> &S = scr[wave];
    if (!shared || qn > kPoolMax) {
        // a longer queue is run by its wavefront alone
        int ns = 0;
        nav_flush<U, HAS_OFFS, false, KSET, SURF>(dau_all + first, cul_all + first, offs, t, base, S, qn,
                                                 ns, lane, nullptr);
        if (!shared) return;
    }
    // sort the queue by class (stable, in place: both entries are read first)
    {
        const bool on0 = lane < qn, on1 = lane + 64 < qn;
        const unsigned int e0 = on0 ? S.queue[lane] : 0u;
        const unsigned int e1 = on1 ? S.queue[lane + 64] : 0u;
        const DaughterRec *dau = dau_all + first;
        const int c0 = on0 ? kind_class<KSET>(dau[e0 >> 10].shape.kind) : -1;
        const int c1 = on1 ? kind_class<KSET>(dau[e1 >> 10].shape.kind) : -1;
        int d0 = 0, d1 = 0, off = 0;
#pragma unroll
        for (int c = 0; c < NK; ++c) {
            const unsigned long long m0 = __builtin_amdgcn_ballot_w64(c0 == c);
            const unsigned long long m1 = __builtin_amdgcn_ballot_w64(c1 == c);
            if (c0 == c) d0 = off + lanes_below(m0);
            if (c1 == c) d1 = off + __popcll(m0) + lanes_below(m1);
            const int n = __popcll(m0) + __popcll(m1);
            if (lane == c) P.cnt[wave][c] = n;
            off += n;
        }
        if (on0) S.pooled.entry[d0] = e0;
        if (on1) S.pooled.entry[d1] = e1;
        if (lane == 0) {
            P.base[wave] = base;
            P.first[wave] = first;
        }
    }
    __syncthreads();
    // per class: each wavefront's share, the pooled count and the number of
    // batches (uniform values)
    int cn[W][NK], tot[NK], nbc[NK], nb = 0;
#pragma unroll
    for (int c = 0; c < NK; ++c) {
        int n = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            cn[w][c] = __builtin_amdgcn_readfirstlane(P.cnt[w][c]);
            n += cn[w][c];
        }
        tot[c] = n;
        nbc[c] = (n + 63) >> 6;
        nb += nbc[c];
    }
    for (int b = wave; b < nb; b += W) {
        // the batch's class and its part within the class
        int c = 0, p = b;
#pragma unroll
        for (int cc = 0; cc < NK - 1; ++cc)
            if (c == cc && p >= nbc[cc]) {
                p -= nbc[cc];
                c = cc + 1;
            }
        const int l = p * 64 + lane;  // the lane's pair within the class
        // the class's pairs run through the wavefronts' sorted queues in
        // order: the owner and the pair's place in its queue
        int own = 0, pos = 0, pre = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            int before = 0, n = 0;
#pragma unroll
            for (int cc = 0; cc < NK; ++cc) {
                if (cc < c) before += cn[w][cc];
                if (cc == c) n = cn[w][cc];
            }
            if (l >= pre && l < pre + n) {
                own = w;
                pos = before + (l - pre);
            }
            pre += n;
        }
        if (l < pre) {
            NavScratch<U> &O = scr[own];
            const unsigned int e = O.pooled.entry[pos];
            const int j = (int)(e & 1023u);
            const int k = (int)(e >> 10);
            const int sl = lds_load(&O.slot_of[j]);
            double x, y, z, ux, uy, uz;
            if (sl != kNoSlot) {
                x = lds_load(&O.x[sl]);
                y = lds_load(&O.y[sl]);
                z = lds_load(&O.z[sl]);
                ux = lds_load(&O.ux[sl]);
                uy = lds_load(&O.uy[sl]);
                uz = lds_load(&O.uz[sl]);
            } else {
                const int64_t i = P.base[own] + j;
                x = t.x[i];
                y = t.y[i];
                z = t.z[i];
                ux = t.ux[i];
                uy = t.uy[i];
                uz = t.uz[i];
            }
            const int f = P.first[own];
            int sid;
            const double s = daughter_dist_out<HAS_OFFS, KSET>(dau_all[f + k], cul_all[f + k], offs, k, x, y,
                                                               z, ux, uy, uz, sid, c);
            O.pooled.key[pos] = step_key(s);
            O.pooled.hit[pos] = hit_pack(k, SURF ? sid : -1);
        }
    }
    __syncthreads();
    // each wavefront merges its own pairs' results
    for (int e0 = 0; e0 < qn; e0 += 64) {
        const int e = e0 + lane;
        if (e < qn) merge_key(S, (int)(S.pooled.entry[e] & 1023u), S.pooled.key[e], S.pooled.hit[e]);
    }
}

// The navigator of the W tiles of a workgroup (wavefront `wave` holds
// `count` tracks from `base` of volume v, whose records start at `first`;
// count may be 0, the wavefront then only taking part in the pooled flush),
// the last flush pooled over the workgroup when `shared`.
template <int U, int W, bool HAS_OFFS, bool HITPT, int KSET>
__device__ __forceinline__ void nav_compact_pooled(const VolumeRec &v, const DaughterRec *__restrict__ dau_all,
                                                   const CullRec *__restrict__ cul_all, int first,
                                                   const double *__restrict__ offs, const TracksDev &t,
                                                   int64_t base, int count, NavScratch<U> *scr,
                                                   PoolInfo<W> &P, bool shared, int wave, int lane,
                                                   double *__restrict__ step, int32_t *__restrict__ hit,
                                                   double *__restrict__ hitpt) {
    int qn = 0;
    if (count > 0)
        qn = nav_compact_core<U, HAS_OFFS, false, KSET, false, false>(v, dau_all + first, cul_all + first, offs,
                                                                     t, base, count, scr[wave], lane);
    pool_flush<U, W, HAS_OFFS, KSET, false>(dau_all, cul_all, offs, t, scr, P, shared, wave, first, base, qn,
                                            lane);
    nav_write<U, HITPT>(scr[wave], t, base, count, lane, step, hit, hitpt);
}

// ---------------------------- compacted navigator safety and localization
// The same queue for the navigator's other two tasks. Safety: a daughter is
// queued for a point when |w| < s_mother + r (its Safety is at least
// |w| - r, so otherwise it cannot go below the mother's, hence not below the
// minimum); the minimum is merged as a 64-bit key like the step (-0 as +0).
// Localization: a daughter is queued for a point inside the mother when
// |w| <= r; the lowest index of a queued daughter that contains the point
// wins (an integer LDS min). The culling tests form w = p - T explicitly, as
// points may lie outside the mother. The sequential loops report -0 as +0
// too, so both forms give the same bits.
__device__ __forceinline__ unsigned long long safety_key(double s) {
    return s == s ? step_key(s) : ~0ull;
}

// Scratch of the compacted safety and localization: the navigator's, plus
// the wavefront's points, which the queued pairs read back from LDS instead
// of global memory (each lane stores its own point; the batches read them
// later in the same wavefront's program order).
template <int U>
struct PointScratch : PointQueue {
    static_assert(U == 1, "one round of 64 points per wavefront");
    double px[64], py[64], pz[64];
};

template <int MODE, bool HAS_OFFS, int KSET, int U>  // MODE 0: safety, 1: locate
__device__ __forceinline__ void point_flush(const DaughterRec *__restrict__ dau,
                                            const CullRec *__restrict__ cul,
                                            const double *__restrict__ offs, PointScratch<U> &S,
                                            int qn, int lane) {
    for (int e0 = 0; e0 < qn; e0 += 64) {
        const int e = e0 + lane;
        if (e < qn) {
            const unsigned int q = S.queue[e];
            const int j = (int)(q & 1023u);
            const int k = (int)(q >> 10);
            const CullRec &Q = cul[k];
            double wx = lds_load(&S.px[j]) - Q.tx, wy = lds_load(&S.py[j]) - Q.ty,
                   wz = lds_load(&S.pz[j]) - Q.tz;
            if (HAS_OFFS) {
                wx -= offs[3 * k + 0];
                wy -= offs[3 * k + 1];
                wz -= offs[3 * k + 2];
            }
            const DaughterRec &D = dau[k];
            const double *R = D.rot;
            const double lx = fma(R[6], wz, fma(R[3], wy, R[0] * wx));
            const double ly = fma(R[7], wz, fma(R[4], wy, R[1] * wx));
            const double lz = fma(R[8], wz, fma(R[5], wy, R[2] * wx));
            if (MODE == 0) {
                const unsigned long long key = safety_key(any_safety<KSET>(D.shape, D.pcon, lx, ly, lz));
                __hip_atomic_fetch_min(&S.key[j], key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
            } else if (any_contains<KSET>(D.shape, D.pcon, lx, ly, lz)) {
                __hip_atomic_fetch_min(&S.hit[j], k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
            }
        }
    }
}

// Safety (MODE 0, out_s) or localization (MODE 1, out_w) of the points
// base + u * 64 + lane (u < U, index below `count` past base). In
// localization mode the key slots hold whether the point is in the mother.
template <int MODE, bool HAS_OFFS, int KSET, int U>
__device__ __forceinline__ void point_compact(const VolumeRec &v, const DaughterRec *__restrict__ dau,
                                              const CullRec *__restrict__ cul,
                                              const double *__restrict__ offs, const TracksDev &t,
                                              int64_t base, int count, PointScratch<U> &S, int lane,
                                              double *__restrict__ out_s,
                                              int32_t *__restrict__ out_w) {
    int qn = 0;
    const int nd = v.nd;
    const int ndp = (nd + kCullChunk - 1) / kCullChunk * kCullChunk;
#pragma unroll 1
    for (int u = 0; u < U; ++u) {
        if (u * 64 >= count) break;
        const int j = u * 64 + lane;
        const bool act = j < count;
        const int64_t i = base + (act ? j : 0);
        const double x = t.x[i], y = t.y[i], z = t.z[i];
        lds_store(&S.px[j], x);
        lds_store(&S.py[j], y);
        lds_store(&S.pz[j], z);
        double reach = 0.0;
        bool in_m = false;
        if (MODE == 0) {
            const double ms = any_safety<KSET>(v.mother, v.pcon, x, y, z);
            lds_store(&S.key[j], safety_key(ms));
            reach = ms;
        } else {
            in_m = any_contains<KSET>(v.mother, v.pcon, x, y, z);
            lds_store(&S.key[j], (unsigned long long)in_m);
            lds_store(&S.hit[j], 0x7fffffff);
        }
        const unsigned long long amask = __builtin_amdgcn_ballot_w64(MODE == 0 ? act : (act && in_m));
        if (amask == 0ull) continue;
        // per-point constants of the expanded test (no offsets): |p|^2, -2 p,
        // and for the safety 2 reach and reach^2; a lane outside amask gets
        // |p|^2 = +inf, so that none of its expanded tests passes and their
        // ballots need no mask (nor do padding records, whose q is -inf)
        double pp = fma(z, z, fma(y, y, x * x));
        if (!((amask >> lane) & 1ull)) pp = __builtin_inf();
        const double mpx = -2.0 * x, mpy = -2.0 * y, mpz = -2.0 * z;
        const double reach2 = 2.0 * reach, rr = reach * reach;
        for (int k0 = 0; k0 < ndp; k0 += kCullChunk) {
            if (qn > kQueueCap - 64 * kCullChunk) {
                point_flush<MODE, HAS_OFFS, KSET, U>(dau, cul, offs, S, qn, lane);
                qn = 0;
            }
            // the chunk's records and offsets, loaded together before its
            // tests (scalar loads; padding records take daughter 0's offsets:
            // they never pass)
            double ctx[kCullChunk], cty[kCullChunk], ctz[kCullChunk], cr[kCullChunk], clim[kCullChunk];
            double cox[kCullChunk], coy[kCullChunk], coz[kCullChunk];
#pragma unroll
            for (int kk = 0; kk < kCullChunk; ++kk) {
                const CullRec &Q = cul[k0 + kk];
                const DaughterRec &D = dau[k0 + kk];
                ctx[kk] = Q.tx;
                cty[kk] = Q.ty;
                ctz[kk] = Q.tz;
                cr[kk] = D.cull_r;
                clim[kk] = HAS_OFFS ? D.cull_r2 : Q.q;
                if (HAS_OFFS) {
                    const int ko = k0 + kk < nd ? k0 + kk : 0;
                    cox[kk] = offs[3 * ko + 0];
                    coy[kk] = offs[3 * ko + 1];
                    coz[kk] = offs[3 * ko + 2];
                }
            }
            unsigned long long cm[kCullChunk];
#pragma unroll
            for (int kk = 0; kk < kCullChunk; ++kk) {
                const int k = k0 + kk;
                bool pass;
                if (HAS_OFFS) {
                    // the centre moves with the offset: |w|^2 formed explicitly
                    const double wx = x - ctx[kk] - cox[kk];
                    const double wy = y - cty[kk] - coy[kk];
                    const double wz = z - ctz[kk] - coz[kk];
                    const double ww = fma(wz, wz, fma(wy, wy, wx * wx));
                    if (MODE == 0) {
                        const double lim = reach + cr[kk];
                        pass = ww < lim * lim;
                    } else {
                        pass = ww <= clim[kk];
                    }
                } else {
                    // |w|^2 - |T|^2 = |p|^2 - 2 p.T against the thresholds less
                    // |T|^2: r^2 - |T|^2 (q, its rounding bound included) for
                    // the containment, (reach + r)^2 - |T|^2 = q + 2 r reach +
                    // reach^2 for a daughter that may be nearer than reach
                    // (reach is at most the mother's bounding radius R for a
                    // point inside the mother, so every term stays within the
                    // (3 R + 2 |T|)^2 that the bound of q covers)
                    const double g = fma(ctz[kk], mpz, fma(cty[kk], mpy, fma(ctx[kk], mpx, pp)));
                    if (MODE == 0)
                        pass = g < fma(cr[kk], reach2, clim[kk]) + rr;
                    else
                        pass = g <= clim[kk];
                }
                // with offsets, lanes outside amask and padding records (k >= nd,
                // whose radius is 0) are masked here
                const unsigned long long bal = __builtin_amdgcn_ballot_w64(pass);
                cm[kk] = HAS_OFFS ? bal & (k < nd ? amask : 0ull) : bal;
            }
#pragma unroll
            for (int kk = 0; kk < kCullChunk; ++kk) {
                const unsigned long long m = cm[kk];
                if (m == 0ull) continue;
                if (__builtin_amdgcn_inverse_ballot_w64(m))
                    S.queue[qn + lanes_below(m)] = ((unsigned int)(k0 + kk) << 10) | (unsigned int)j;
                qn += __popcll(m);
            }
        }
    }
    point_flush<MODE, HAS_OFFS, KSET, U>(dau, cul, offs, S, qn, lane);
#pragma unroll 1
    for (int u = 0; u < U; ++u) {
        const int j = u * 64 + lane;
        if (j < count) {
            const int64_t o = base + j;
            if (MODE == 0) {
                out_s[o] = key_step(lds_load(&S.key[j]));
            } else {
                const int w = lds_load(&S.hit[j]);
                out_w[o] = lds_load(&S.key[j]) == 0ull ? -2 : (w != 0x7fffffff ? w : -1);
            }
        }
    }
}

// ------------------------------------------ navigator safety and locate
// The navigator's other two per-track tasks (section 3), sequential form
// with every daughter evaluated (culling off; the culled kernels take the
// compacted form above).
template <bool HAS_OFFS, int KSET = kSetAll>
__device__ __forceinline__ double nav_safety(const VolumeRec &v, const DaughterRec *__restrict__ dau,
                                             const CullRec *__restrict__ cul,
                                             const double *__restrict__ offs, double x, double y,
                                             double z) {
    double best = any_safety<KSET>(v.mother, v.pcon, x, y, z);
    const int nd = v.nd;
    for (int k = 0; k < nd; ++k) {
        const CullRec &Q = cul[k];
        double wx = x - Q.tx, wy = y - Q.ty, wz = z - Q.tz;
        if (HAS_OFFS) {
            wx -= offs[3 * k + 0];
            wy -= offs[3 * k + 1];
            wz -= offs[3 * k + 2];
        }
        const DaughterRec &D = dau[k];
        const double *R = D.rot;
        const double lx = fma(R[6], wz, fma(R[3], wy, R[0] * wx));
        const double ly = fma(R[7], wz, fma(R[4], wy, R[1] * wx));
        const double lz = fma(R[8], wz, fma(R[5], wy, R[2] * wx));
        best = fmin(best, any_safety<KSET>(D.shape, D.pcon, lx, ly, lz));
    }
    return best == 0.0 ? 0.0 : best;  // -0 reported as +0
}

// Daughter holding the point (lowest index), -1 for the mother's own part,
// -2 outside the mother.
template <bool HAS_OFFS, int KSET = kSetAll>
__device__ __forceinline__ int nav_locate(const VolumeRec &v, const DaughterRec *__restrict__ dau,
                                          const CullRec *__restrict__ cul,
                                          const double *__restrict__ offs, double x, double y,
                                          double z) {
    int where = any_contains<KSET>(v.mother, v.pcon, x, y, z) ? -1 : -2;
    const int nd = v.nd;
    for (int k = 0; k < nd; ++k) {
        if (__ballot(where == -1) == 0) break;  // every lane placed
        const CullRec &Q = cul[k];
        double wx = x - Q.tx, wy = y - Q.ty, wz = z - Q.tz;
        if (HAS_OFFS) {
            wx -= offs[3 * k + 0];
            wy -= offs[3 * k + 1];
            wz -= offs[3 * k + 2];
        }
        const DaughterRec &D = dau[k];
        const double *R = D.rot;
        const double lx = fma(R[6], wz, fma(R[3], wy, R[0] * wx));
        const double ly = fma(R[7], wz, fma(R[4], wy, R[1] * wx));
        const double lz = fma(R[8], wz, fma(R[5], wy, R[2] * wx));
        const bool in = any_contains<KSET>(D.shape, D.pcon, lx, ly, lz);
        where = (where == -1 && in) ? k : where;
    }
    return where;
}

}  // namespace gn

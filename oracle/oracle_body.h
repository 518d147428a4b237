/*
 * Body of the CPU oracle, instantiated once per real type by oracle.c with
 *   R      the real type (double or long double),
 *   FN(n)  the name mangler (n##_d or n##_ld).
 * <tgmath.h> makes sqrt/fabs resolve to the variant of R.
 *
 * Every query is written as its plain definition (see oracle.c's header):
 * membership tests, Euclidean distances to the profile's edges, and the
 * intersection of the flight line with the solid as a set of intervals.
 */

/* ---------------------------------------------------------------- Contains
 * Closed-set membership test ("inside/outside checks", section 3.1).      */
static int FN(in_wedge)(R phi1, R dphi, R x, R y);
static int FN(segment)(int kind, const double *par, int *base, R *phi1, R *dphi);
static int FN(pcon_in_profile)(const double *par, R r, R z);

static int FN(contains)(int kind, const double *par, R x, R y, R z)
{
    int base;
    R phi1, dphi;
    if (FN(segment)(kind, par, &base, &phi1, &dphi) && !FN(in_wedge)(phi1, dphi, x, y)) return 0;
    if (kind == OR_TUBS) kind = OR_TUBE;           /* in the range (or uncut): the base solid */
    if (kind == OR_CONS) kind = OR_CONE;
    if (kind == OR_PCON) return FN(pcon_in_profile)(par, sqrt(x * x + y * y), z);
    if (kind == OR_BOX)
        return fabs(x) <= (R)par[0] && fabs(y) <= (R)par[1] && fabs(z) <= (R)par[2];
    if (kind == OR_TUBE) {
        R r = sqrt(x * x + y * y);
        return fabs(z) <= (R)par[2] && r >= (R)par[0] && r <= (R)par[1];
    }
    if (kind == OR_CONE) {
        R dz = par[0];
        if (fabs(z) > dz) return 0;
        R f = (z + dz) / (2 * dz);                    /* 0 at -dz, 1 at +dz */
        R rin = (R)par[1] + ((R)par[3] - (R)par[1]) * f;
        R rout = (R)par[2] + ((R)par[4] - (R)par[2]) * f;
        R r = sqrt(x * x + y * y);
        return r >= rin && r <= rout;
    }
    return -1;
}

/* -------------------------------------------------------------- Segments
 * The segmented tube and cone (section 3.1 names the segmented forms of tube
 * and cone among the shapes ported) and the polycone: a solid of revolution
 * cut to the azimuth range [phi1, phi1 + dphi], the z axis included. The
 * leading parameters of TUBS and CONS are the base kind's (TUBS: rmin rmax
 * dz phi1 dphi; CONS: dz rmin1 rmax1 rmin2 rmax2 phi1 dphi); the polycone's
 * range leads its parameters. Angles in radians. dphi at or above 2 pi (as
 * a double) leaves the solid uncut. Returns 1 for a cut solid, with the
 * kind of its uncut base.                                                  */
static int FN(segment)(int kind, const double *par, int *base, R *phi1, R *dphi)
{
    if (kind == OR_TUBS) { *base = OR_TUBE; *phi1 = par[3]; *dphi = par[4]; }
    else if (kind == OR_CONS) { *base = OR_CONE; *phi1 = par[5]; *dphi = par[6]; }
    else if (kind == OR_PCON) { *base = OR_PCON; *phi1 = par[0]; *dphi = par[1]; }
    else return 0;
    return *dphi < (R)OR_FULL_TURN;
}

/* -------------------------------------------------------------- Polycone
 * A sequence of connected cone and tube sections (section 3.1):
 * par = {phi1, dphi, nz, z_0, rmin_0, rmax_0, ..., z_{nz-1}, rmin_{nz-1},
 * rmax_{nz-1}}, 2 <= nz <= OR_PCON_MAX, z strictly increasing; between two
 * consecutive planes both radii vary linearly in z. In its (r, z) half-plane
 * the solid's profile is the polygon up the outer radii and back down the
 * inner ones.                                                             */
static int FN(pcon_planes)(const double *par, R *z, R *rin, R *rout)
{
    int n = (int)par[2];
    for (int j = 0; j < n; ++j) {
        z[j] = par[3 + 3 * j];
        rin[j] = par[4 + 3 * j];
        rout[j] = par[5 + 3 * j];
    }
    return n;
}

static int FN(pcon_in_profile)(const double *par, R r, R zz)
{
    R z[OR_PCON_MAX], rin[OR_PCON_MAX], rout[OR_PCON_MAX];
    int n = FN(pcon_planes)(par, z, rin, rout);
    for (int j = 0; j + 1 < n; ++j) {
        if (zz < z[j] || zz > z[j + 1]) continue;
        R f = (zz - z[j]) / (z[j + 1] - z[j]);
        if (r >= rin[j] + (rin[j + 1] - rin[j]) * f && r <= rout[j] + (rout[j + 1] - rout[j]) * f)
            return 1;
    }
    return 0;
}

/* Azimuth of (x, y) in the closed range [phi1, phi1 + dphi] modulo 2 pi;
 * the axis has every azimuth. */
static int FN(in_wedge)(R phi1, R dphi, R x, R y)
{
    if (x == 0 && y == 0) return 1;
    R a = atan2(y, x) - phi1;
    a -= (R)OR_TWO_PI * floor(a / (R)OR_TWO_PI);   /* into [0, 2 pi] */
    return a <= dphi;
}

/* ------------------------------------------------------------------ Safety
 * Euclidean distance from p to the boundary of the shape, "the minimum
 * distance to any boundary" (section 3.1).                                 */

/* Distance from (u, v) to the segment (u0, v0)-(u1, v1) in a plane. */
static R FN(seg_dist)(R u, R v, R u0, R v0, R u1, R v1)
{
    R eu = u1 - u0, ev = v1 - v0;
    R wu = u - u0, wv = v - v0;
    R ee = eu * eu + ev * ev;
    R t = 0;
    if (ee > 0) {
        t = (wu * eu + wv * ev) / ee;
        if (t < 0) t = 0;
        if (t > 1) t = 1;
    }
    R du = wu - t * eu, dv = wv - t * ev;
    return sqrt(du * du + dv * dv);
}

/* Profile quadrilateral of a tube or cone in its (r, z) half-plane:
 *   A(rin1, -dz) B(rout1, -dz) C(rout2, +dz) D(rin2, +dz). */
static int FN(profile)(int kind, const double *par, R *rin1, R *rout1, R *rin2, R *rout2, R *dz)
{
    if (kind == OR_TUBE || kind == OR_TUBS) {
        *rin1 = *rin2 = par[0];
        *rout1 = *rout2 = par[1];
        *dz = par[2];
        return 1;
    }
    if (kind == OR_CONE || kind == OR_CONS) {
        *dz = par[0];
        *rin1 = par[1]; *rout1 = par[2];
        *rin2 = par[3]; *rout2 = par[4];
        return 1;
    }
    return 0;
}

/* Distance from (u, z) to the closed quadrilateral (0 inside or on it). */
static R FN(quad_dist)(R u, R z, R rin1, R rout1, R rin2, R rout2, R dz)
{
    if (fabs(z) <= dz) {
        R f = (z + dz) / (2 * dz);
        if (u >= rin1 + (rin2 - rin1) * f && u <= rout1 + (rout2 - rout1) * f) return 0;
    }
    R best = FN(seg_dist)(u, z, rin1, -dz, rout1, -dz);
    R s = FN(seg_dist)(u, z, rout1, -dz, rout2, dz);
    if (s < best) best = s;
    s = FN(seg_dist)(u, z, rout2, dz, rin2, dz);
    if (s < best) best = s;
    s = FN(seg_dist)(u, z, rin2, dz, rin1, -dz);
    if (s < best) best = s;
    return best;
}

/* Polycone profile: the smallest distance from (u, z) to its edges (the two
 * end edges, the outer edges and the inner edges; with `axis` 0 an inner
 * edge lying on the axis is skipped, as it bounds no surface of the uncut
 * solid), and 0 for a point of the polygon when `solid` is set. */
static R FN(pcon_edges_dist)(const double *par, R u, R zz, int axis, int solid)
{
    if (solid && FN(pcon_in_profile)(par, u, zz)) return 0;
    R z[OR_PCON_MAX], rin[OR_PCON_MAX], rout[OR_PCON_MAX];
    int n = FN(pcon_planes)(par, z, rin, rout);
    R best = FN(seg_dist)(u, zz, rin[0], z[0], rout[0], z[0]);
    R s = FN(seg_dist)(u, zz, rin[n - 1], z[n - 1], rout[n - 1], z[n - 1]);
    if (s < best) best = s;
    for (int j = 0; j + 1 < n; ++j) {
        s = FN(seg_dist)(u, zz, rout[j], z[j], rout[j + 1], z[j + 1]);
        if (s < best) best = s;
        if (!axis && rin[j] == 0 && rin[j + 1] == 0) continue;
        s = FN(seg_dist)(u, zz, rin[j], z[j], rin[j + 1], z[j + 1]);
        if (s < best) best = s;
    }
    return best;
}

/* Distance from p to the flat face of a segment at azimuth phi: the profile
 * polygon laid in the half-plane at that azimuth. With u the coordinate
 * along the half-plane's direction (cos phi, sin phi, 0) and v the distance
 * from its plane, it is sqrt(v^2 + dist((u, z), polygon)^2). */
static R FN(face_dist)(int kind, const double *par, R phi, R x, R y, R z)
{
    R c = cos(phi), sn = sin(phi);
    R u = c * x + sn * y, v = -sn * x + c * y;
    R q;
    if (kind == OR_PCON) {
        q = FN(pcon_edges_dist)(par, u, z, 1, 1);
    } else {
        R rin1 = 0, rout1 = 0, rin2 = 0, rout2 = 0, dz = 0;
        FN(profile)(kind, par, &rin1, &rout1, &rin2, &rout2, &dz);
        q = FN(quad_dist)(u, z, rin1, rout1, rin2, rout2, dz);
    }
    return sqrt(v * v + q * q);
}

static R FN(safety)(int kind, const double *par, R x, R y, R z)
{
    int base;
    R phi1, dphi;
    if (FN(segment)(kind, par, &base, &phi1, &dphi)) {
        /* The boundary is the base's surfaces within the azimuth range plus
         * the two faces. For p in the range the nearest point of the base's
         * surfaces has p's own azimuth, so it is the base's Safety; for p
         * outside the range it lies on the edge of a face (the face distance
         * covers it). */
        R best = INFINITY;
        if (FN(in_wedge)(phi1, dphi, x, y))
            best = base == OR_PCON ? FN(pcon_edges_dist)(par, sqrt(x * x + y * y), z, 0, 0)
                                   : FN(safety)(base, par, x, y, z);
        R s = FN(face_dist)(kind, par, phi1, x, y, z);
        if (s < best) best = s;
        s = FN(face_dist)(kind, par, phi1 + dphi, x, y, z);
        if (s < best) best = s;
        return best;
    }
    /* uncut polycone: a solid of revolution, so as for tube and cone the
     * planar distance from (r, z) to the profile's edges */
    if (kind == OR_PCON) return FN(pcon_edges_dist)(par, sqrt(x * x + y * y), z, 0, 0);
    if (kind == OR_BOX) {
        R ax = fabs(x), ay = fabs(y), az = fabs(z);
        R dx = par[0], dy = par[1], dz = par[2];
        if (FN(contains)(kind, par, x, y, z)) {
            /* inside: nearest face */
            R s = dx - ax;
            if (dy - ay < s) s = dy - ay;
            if (dz - az < s) s = dz - az;
            return s;
        }
        /* outside: distance to the solid (equal to the distance to its
         * surface), per-axis excess */
        R ex = ax > dx ? ax - dx : 0, ey = ay > dy ? ay - dy : 0, ez = az > dz ? az - dz : 0;
        return sqrt(ex * ex + ey * ey + ez * ez);
    }
    /* Tube and cone are solids of revolution: the nearest boundary point
     * lies in p's own half-plane, so the distance is the planar distance
     * from (r, z) to the edges of the profile quadrilateral
     *   A(rin1, -dz) B(rout1, -dz) C(rout2, +dz) D(rin2, +dz).
     * An edge on the axis (r = 0) bounds no surface and is skipped. */
    R rin1, rout1, rin2, rout2, dz;
    if (!FN(profile)(kind, par, &rin1, &rout1, &rin2, &rout2, &dz)) return -1;
    R r = sqrt(x * x + y * y);
    R best = FN(seg_dist)(r, z, rin1, -dz, rout1, -dz);              /* bottom AB */
    R s = FN(seg_dist)(r, z, rout1, -dz, rout2, dz);                  /* outer  BC */
    if (s < best) best = s;
    s = FN(seg_dist)(r, z, rout2, dz, rin2, dz);                      /* top    CD */
    if (s < best) best = s;
    if (!(rin1 == 0 && rin2 == 0)) {
        s = FN(seg_dist)(r, z, rin2, dz, rin1, -dz);                  /* inner  DA */
        if (s < best) best = s;
    }
    return best;
}

/* ------------------------------------------------ line-solid intersection
 * The flight line p + t d meets a solid in a set of closed t-intervals.    */
typedef struct { R lo, hi; } FN(ival);

/* {t : |z0 + t uz| <= h}. Returns 0 if empty. */
static int FN(slab)(R z0, R uz, R h, R *lo, R *hi)
{
    if (uz == 0) {
        if (fabs(z0) <= h) { *lo = -INFINITY; *hi = INFINITY; return 1; }
        return 0;
    }
    R t1 = (-h - z0) / uz, t2 = (h - z0) / uz;
    *lo = t1 < t2 ? t1 : t2;
    *hi = t1 < t2 ? t2 : t1;
    return 1;
}

/* Is the line point at t inside the closed nappe solid
 * N(a, b) = { sqrt(x^2 + y^2) <= a + b z } ? */
static int FN(in_nappe)(R a, R b, const R *p, const R *d, R t)
{
    R x = p[0] + t * d[0], y = p[1] + t * d[1], z = p[2] + t * d[2];
    return sqrt(x * x + y * y) <= a + b * z;
}

/* On the boundary of N the squared form
 * f(t) = (a + b z(t))^2 - (x(t)^2 + y(t)^2) vanishes, so the line's crossings
 * of the nappe are among the real roots of this quadratic (ascending; the
 * mirror nappe a + b z < 0 contributes roots too). */
static int FN(nappe_roots)(R a, R b, const R *p, const R *d, R *roots)
{
    R w0 = a + b * p[2];
    R wz = b * d[2];
    R qa = wz * wz - (d[0] * d[0] + d[1] * d[1]);
    R qb = 2 * (w0 * wz - (p[0] * d[0] + p[1] * d[1]));
    R qc = w0 * w0 - (p[0] * p[0] + p[1] * p[1]);
    int nr = 0;
    if (qa == 0) {
        if (qb != 0) roots[nr++] = -qc / qb;
    } else {
        R disc = qb * qb - 4 * qa * qc;
        if (disc == 0) {
            roots[nr++] = -qb / (2 * qa);
        } else if (disc > 0) {
            R sq = sqrt(disc);
            R q = -(qb + (qb >= 0 ? sq : -sq)) / 2;
            R r1 = q / qa, r2 = qc / q;
            roots[0] = r1 < r2 ? r1 : r2;
            roots[1] = r1 < r2 ? r2 : r1;
            nr = 2;
        }
    }
    return nr;
}

/* Line intersected with the convex solid N(a, b): a single closed interval
 * (maybe unbounded) or empty (returns 0). Membership is decided by testing
 * one interior point of every piece between the roots (which also rejects
 * the mirror nappe). */
static int FN(line_nappe)(R a, R b, const R *p, const R *d, R *lo, R *hi)
{
    R roots[2];
    int nr = FN(nappe_roots)(a, b, p, d, roots);
    if (nr == 0) {
        if (FN(in_nappe)(a, b, p, d, 0)) { *lo = -INFINITY; *hi = INFINITY; return 1; }
        return 0;
    }
    /* Pieces between consecutive roots, each with one interior sample; a
     * root on its own is a piece too (a touching point). */
    R plo[5], phi[5], smp[5];
    int np = 0;
    R first = roots[0], last = roots[nr - 1];
    plo[np] = -INFINITY; phi[np] = first; smp[np] = first - (1 + fabs(first)); np++;
    plo[np] = first; phi[np] = first; smp[np] = first; np++;
    if (nr == 2) {
        plo[np] = first; phi[np] = last; smp[np] = first + (last - first) / 2; np++;
        plo[np] = last; phi[np] = last; smp[np] = last; np++;
    }
    plo[np] = last; phi[np] = INFINITY; smp[np] = last + (1 + fabs(last)); np++;
    int found = 0;
    for (int i = 0; i < np; ++i) {
        if (!FN(in_nappe)(a, b, p, d, smp[i])) continue;
        if (!found) { *lo = plo[i]; *hi = phi[i]; found = 1; }
        else {
            if (plo[i] < *lo) *lo = plo[i];
            if (phi[i] > *hi) *hi = phi[i];
        }
    }
    return found;
}

/* Intersect [lo, hi] with [a, b]; returns 0 if empty. */
static int FN(cap)(R *lo, R *hi, R a, R b)
{
    if (a > *lo) *lo = a;
    if (b < *hi) *hi = b;
    return *lo <= *hi;
}

static int FN(line_segment)(int kind, const double *par, const R *p, const R *d, FN(ival) *out);

/* Line intersected with the shape: closed intervals, ascending (at most
 * OR_MAX_IVAL).
 * Box: the three slabs intersected (Kay-Kajiya).
 * Tube and cone: (z-slab  and  outer nappe solid)  minus  the open inner
 * nappe solid {r < rin(z)}, which is empty when both inner radii are 0.
 * Segments and polycones: see line_segment.                                */
static int FN(line_shape)(int kind, const double *par, const R *p, const R *d, FN(ival) *out)
{
    R lo, hi, a, b;
    int base;
    R phi1, dphi;
    if (FN(segment)(kind, par, &base, &phi1, &dphi) || kind == OR_PCON)
        return FN(line_segment)(kind, par, p, d, out);
    if (kind == OR_TUBS || kind == OR_CONS)      /* uncut: the base solid */
        kind = kind == OR_TUBS ? OR_TUBE : OR_CONE;
    if (kind == OR_BOX) {
        lo = -INFINITY; hi = INFINITY;
        for (int i = 0; i < 3; ++i) {
            if (!FN(slab)(p[i], d[i], (R)par[i], &a, &b)) return 0;
            if (!FN(cap)(&lo, &hi, a, b)) return 0;
        }
        out[0].lo = lo; out[0].hi = hi;
        return 1;
    }
    R dz, ao, bo, ai, bi;
    int hole;
    if (kind == OR_TUBE) {
        dz = par[2];
        ao = par[1]; bo = 0;
        ai = par[0]; bi = 0;
        hole = par[0] != 0;
    } else if (kind == OR_CONE) {
        dz = par[0];
        /* radius at z is linear: r(z) = a + b z with r(-dz) = r1, r(dz) = r2 */
        ao = ((R)par[2] + (R)par[4]) / 2; bo = ((R)par[4] - (R)par[2]) / (2 * dz);
        ai = ((R)par[1] + (R)par[3]) / 2; bi = ((R)par[3] - (R)par[1]) / (2 * dz);
        hole = !(par[1] == 0 && par[3] == 0);
    } else {
        return 0;
    }
    if (!FN(slab)(p[2], d[2], dz, &lo, &hi)) return 0;
    if (!FN(line_nappe)(ao, bo, p, d, &a, &b)) return 0;
    if (!FN(cap)(&lo, &hi, a, b)) return 0;
    if (!hole || !FN(line_nappe)(ai, bi, p, d, &a, &b)) {
        out[0].lo = lo; out[0].hi = hi;
        return 1;
    }
    /* [lo, hi] minus the open interval (a, b) */
    int n = 0;
    if (lo <= a) { out[n].lo = lo; out[n].hi = hi < a ? hi : a; n++; }
    if (hi >= b) { out[n].lo = lo > b ? lo : b; out[n].hi = hi; n++; }
    return n;
}

/* A segment's or polycone's boundary lies on its z planes, on the nappes
 * through the profile's slanted edges and (when cut) on the two planes
 * through the axis at azimuths phi1 and phi1 + dphi, so the line's intervals
 * in the solid end at crossings of these surfaces. Split the line at every
 * crossing, test membership (Contains) at one interior point of each open
 * piece and at each crossing, and join neighbouring pieces that belong.
 * Membership is constant on a piece, and the solid is closed: a crossing
 * next to a piece that belongs belongs too. Crossings of a whole plane, of
 * a nappe beyond its section or of a mirror nappe only split a piece
 * needlessly.                                                             */
static int FN(line_segment)(int kind, const double *par, const R *p, const R *d, FN(ival) *out)
{
    int base;
    R phi1 = 0, dphi = 0;
    int cut = FN(segment)(kind, par, &base, &phi1, &dphi);
    /* the profile as a list of planes (z, rin, rout) */
    R z[OR_PCON_MAX], rin[OR_PCON_MAX], rout[OR_PCON_MAX];
    int np = 2;
    if (kind == OR_PCON) {
        np = FN(pcon_planes)(par, z, rin, rout);
    } else {
        R dz = 0;
        FN(profile)(kind, par, &rin[0], &rout[0], &rin[1], &rout[1], &dz);
        z[0] = -dz;
        z[1] = dz;
    }
    R t[5 * OR_PCON_MAX];                       /* np planes + 4 per section + 2 */
    int m = 0;
    if (d[2] != 0)
        for (int j = 0; j < np; ++j) t[m++] = (z[j] - p[2]) / d[2];
    /* nappes r = a + b z through each section's slanted edges */
    for (int j = 0; j + 1 < np; ++j) {
        R h = z[j + 1] - z[j];
        R bo = (rout[j + 1] - rout[j]) / h, bi = (rin[j + 1] - rin[j]) / h;
        m += FN(nappe_roots)(rout[j] - bo * z[j], bo, p, d, t + m);
        if (!(rin[j] == 0 && rin[j + 1] == 0)) m += FN(nappe_roots)(rin[j] - bi * z[j], bi, p, d, t + m);
    }
    for (int i = 0; cut && i < 2; ++i) {
        R ph = i == 0 ? phi1 : phi1 + dphi;
        R nx = -sin(ph), ny = cos(ph);             /* normal of the plane at ph */
        R nd = nx * d[0] + ny * d[1];
        if (nd != 0) t[m++] = -(nx * p[0] + ny * p[1]) / nd;
    }
    /* sort ascending, drop repeats */
    for (int i = 1; i < m; ++i)
        for (int j = i; j > 0 && t[j] < t[j - 1]; --j) { R x = t[j]; t[j] = t[j - 1]; t[j - 1] = x; }
    int u = 0;
    for (int i = 0; i < m; ++i)
        if (u == 0 || t[i] != t[u - 1]) t[u++] = t[i];
    m = u;
#define OR_IN_AT(tt) FN(contains)(kind, par, p[0] + (tt) * d[0], p[1] + (tt) * d[1], p[2] + (tt) * d[2])
    if (m == 0) {
        if (!OR_IN_AT(0)) return 0;
        out[0].lo = -INFINITY; out[0].hi = INFINITY;
        return 1;
    }
    /* open pieces 0..m (piece i lies between t[i-1] and t[i]) */
    int piece[5 * OR_PCON_MAX + 1];
    piece[0] = OR_IN_AT(t[0] - (1 + fabs(t[0])));
    for (int i = 1; i < m; ++i) piece[i] = OR_IN_AT(t[i - 1] + (t[i] - t[i - 1]) / 2);
    piece[m] = OR_IN_AT(t[m - 1] + (1 + fabs(t[m - 1])));
    /* walk the pieces and crossings in order; every run of members holds a
     * crossing, so there are at most m runs */
    int n = 0, open = piece[0];
    if (open) out[0].lo = -INFINITY;
    for (int i = 0; i < m; ++i) {                 /* crossing i, then piece i + 1 */
        int at = open || piece[i + 1] || OR_IN_AT(t[i]);
        if (at && !open) out[n].lo = t[i];
        open = piece[i + 1];
        if (at && !open) out[n++].hi = t[i];
    }
    if (open) out[n++].hi = INFINITY;
#undef OR_IN_AT
    return n;
}

/* -------------------------------------------- DistFromOutside / Inside
 * Distance along the line of flight to enter the shape / to leave it
 * (section 3.1). A point already inside has DistFromOutside 0; a point
 * outside has DistFromInside 0. A line that never enters gives OR_BIG.  */
static R FN(dist_out)(int kind, const double *par, const R *p, const R *d)
{
    if (FN(contains)(kind, par, p[0], p[1], p[2])) return 0;
    FN(ival) iv[OR_MAX_IVAL];
    int n = FN(line_shape)(kind, par, p, d, iv);
    R best = OR_BIG;
    for (int i = 0; i < n; ++i) {
        if (iv[i].hi < 0) continue;
        R t = iv[i].lo > 0 ? iv[i].lo : 0;
        if (t < best) best = t;
    }
    return best;
}

static R FN(dist_in)(int kind, const double *par, const R *p, const R *d)
{
    if (!FN(contains)(kind, par, p[0], p[1], p[2])) return 0;
    FN(ival) iv[OR_MAX_IVAL];
    int n = FN(line_shape)(kind, par, p, d, iv);
    for (int i = 0; i < n; ++i)
        if (iv[i].lo <= 0 && iv[i].hi >= 0) return iv[i].hi < OR_BIG ? iv[i].hi : OR_BIG;
    return 0;
}

/* --------------------------------------------------------------- exports */
void FN(or_shape_query)(int kind, const double *par, int query, int64_t n,
                        const double *x, const double *y, const double *z,
                        const double *ux, const double *uy, const double *uz,
                        double *out_val, uint8_t *out_in)
{
    for (int64_t i = 0; i < n; ++i) {
        R p[3] = { x[i], y[i], z[i] };
        if (query == OR_CONTAINS) {
            out_in[i] = (uint8_t)FN(contains)(kind, par, p[0], p[1], p[2]);
        } else if (query == OR_SAFETY) {
            out_val[i] = (double)FN(safety)(kind, par, p[0], p[1], p[2]);
        } else {
            R d[3] = { ux[i], uy[i], uz[i] };
            out_val[i] = (double)(query == OR_DIST_IN ? FN(dist_in)(kind, par, p, d)
                                                      : FN(dist_out)(kind, par, p, d));
        }
    }
}

/* ------------------------------------------------------------ Navigator
 * Fig. 1: the step to the next boundary is the smaller of the mother's
 * distFromInside and, over the daughters, distFromOutside taken in each
 * daughter's own frame; the hit volume is the one attaining it (-1 for the
 * mother). Daughter k places its frame at q -> R_k q + T_k + delta_k, so a
 * mother-frame point p maps back to R_k^T (p - T_k - delta_k).
 * Ties: mother first, then the lowest daughter index (strict <).
 * Also returns the gap between the two smallest candidates.              */
typedef struct {
    int mother_kind;
    const double *mother_par;     /* OR_NPAR */
    int nd;
    const int32_t *kinds;         /* nd */
    const double *pars;           /* nd x OR_NPAR */
    const double *rots;           /* nd x 9, row-major R */
    const double *trs;            /* nd x 3 */
} FN(vol);

static R FN(navigate1)(const FN(vol) *v, const R *p, const R *d, const R *offs,
                       int32_t *hit, R *gap)
{
    R best = FN(dist_in)(v->mother_kind, v->mother_par, p, d);
    R second = OR_BIG * 2;
    int32_t h = -1;
    for (int k = 0; k < v->nd; ++k) {
        const double *rm = v->rots + 9 * k;
        R w[3];
        for (int i = 0; i < 3; ++i)
            w[i] = p[i] - (R)v->trs[3 * k + i] - (offs ? offs[3 * k + i] : 0);
        R pl[3], dl[3];
        for (int j = 0; j < 3; ++j) {           /* (R^T w)_j = sum_i R_ij w_i */
            pl[j] = (R)rm[0 + j] * w[0] + (R)rm[3 + j] * w[1] + (R)rm[6 + j] * w[2];
            dl[j] = (R)rm[0 + j] * d[0] + (R)rm[3 + j] * d[1] + (R)rm[6 + j] * d[2];
        }
        R s = FN(dist_out)(v->kinds[k], v->pars + OR_NPAR * k, pl, dl);
        if (s < best) { second = best; best = s; h = k; }
        else if (s < second) second = s;
    }
    *hit = h;
    if (gap) *gap = second - best;
    return best;
}

void FN(or_navigate)(int mother_kind, const double *mother_par, int nd,
                     const int32_t *kinds, const double *pars, const double *rots,
                     const double *trs, const double *offsets, int64_t n,
                     const double *x, const double *y, const double *z,
                     const double *ux, const double *uy, const double *uz,
                     double *step, int32_t *hit, double *gap)
{
    FN(vol) v = { mother_kind, mother_par, nd, kinds, pars, rots, trs };
    R offs[3 * OR_MAX_DAUGHTERS];
    if (offsets)
        for (int i = 0; i < 3 * nd; ++i) offs[i] = offsets[i];
    for (int64_t i = 0; i < n; ++i) {
        R p[3] = { x[i], y[i], z[i] }, d[3] = { ux[i], uy[i], uz[i] };
        R g;
        step[i] = (double)FN(navigate1)(&v, p, d, offsets ? offs : 0, hit + i, &g);
        if (gap) gap[i] = (double)g;
    }
}

/* --------------------------------------------- adjoint reference (FD)
 * Central finite differences of phi = gs * s + gh . (o + s d), with s the
 * navigator step, with respect to the origin o, the direction d and the
 * offset delta of the hit daughter. A track is flagged non-smooth (mask 0)
 * when the runner-up gap is below min_gap, when any perturbation changes the
 * hit volume, when the forward and backward one-sided differences disagree
 * by more than kink_tol (a kink within the stencil), or when the central
 * differences at h and 2h disagree by more than 3 * fd_tol (the central
 * difference's own error is about a third of that disagreement).          */
static R FN(phi)(const FN(vol) *v, const R *o, const R *d, const R *offs, R gs, const R *gh,
                 int32_t *hit)
{
    R s = FN(navigate1)(v, o, d, offs, hit, 0);
    return gs * s + gh[0] * (o[0] + s * d[0]) + gh[1] * (o[1] + s * d[1]) + gh[2] * (o[2] + s * d[2]);
}

void FN(or_navigate_fd)(int mother_kind, const double *mother_par, int nd,
                        const int32_t *kinds, const double *pars, const double *rots,
                        const double *trs, const double *offsets, int64_t n,
                        const double *x, const double *y, const double *z,
                        const double *ux, const double *uy, const double *uz,
                        const double *gstep, const double *ghit, double h,
                        double min_gap, double kink_tol, double fd_tol,
                        double *g_o, double *g_d, double *g_off, int32_t *hit_out,
                        uint8_t *mask)
{
    FN(vol) v = { mother_kind, mother_par, nd, kinds, pars, rots, trs };
    R offs[3 * OR_MAX_DAUGHTERS];
    for (int i = 0; i < 3 * nd; ++i) offs[i] = offsets ? offsets[i] : 0;
    for (int64_t i = 0; i < n; ++i) {
        R o[3] = { x[i], y[i], z[i] }, d[3] = { ux[i], uy[i], uz[i] };
        R gh[3] = { ghit ? ghit[i] : 0, ghit ? ghit[n + i] : 0, ghit ? ghit[2 * n + i] : 0 };
        R gs = gstep ? gstep[i] : 0;
        int32_t h0;
        R gap;
        FN(navigate1)(&v, o, d, offs, &h0, &gap);
        hit_out[i] = h0;
        int ok = gap >= min_gap;
        R phi0 = FN(phi)(&v, o, d, offs, gs, gh, &h0);
        R grad[9] = { 0 };
        int ndof = h0 >= 0 ? 9 : 6;
        for (int j = 0; j < ndof; ++j) {
            R val[4];
            const R mult[4] = { 1, -1, 2, -2 };
            for (int m = 0; m < 4; ++m) {
                R oo[3] = { o[0], o[1], o[2] }, dd[3] = { d[0], d[1], d[2] };
                R *target = j < 3 ? &oo[j] : j < 6 ? &dd[j - 3] : &offs[3 * h0 + (j - 6)];
                R keep = *target;
                *target = keep + mult[m] * (R)h;
                int32_t hh;
                val[m] = FN(phi)(&v, oo, dd, offs, gs, gh, &hh);
                *target = keep;
                if (hh != h0) ok = 0;
            }
            R c1 = (val[0] - val[1]) / (2 * (R)h);
            R c2 = (val[2] - val[3]) / (4 * (R)h);
            R dp = (val[0] - phi0) / (R)h, dm = (phi0 - val[1]) / (R)h;
            R scale = fabs(c1) > 1 ? fabs(c1) : 1;
            if (fabs(dp - dm) > kink_tol * scale) ok = 0;
            if (fabs(c1 - c2) > 3 * fd_tol * scale) ok = 0;
            grad[j] = c1;
        }
        for (int j = 0; j < 3; ++j) {
            g_o[j * n + i] = (double)grad[j];
            g_d[j * n + i] = (double)grad[3 + j];
            g_off[j * n + i] = (double)grad[6 + j];
        }
        mask[i] = (uint8_t)ok;
    }
}

/* ------------------------------------------- navigator safety and locate
 * The navigator's other two tasks (section 3): the safe distance to the
 * boundaries of the volume — the smaller of the mother's Safety and every
 * daughter's Safety taken in the daughter's frame — and localization: the
 * daughter holding the point (lowest index), -1 for the mother's own part,
 * -2 for a point outside the mother.                                      */
static void FN(local_point)(const FN(vol) *v, int k, const R *p, const R *offs, R *pl)
{
    const double *rm = v->rots + 9 * k;
    R w[3];
    for (int i = 0; i < 3; ++i)
        w[i] = p[i] - (R)v->trs[3 * k + i] - (offs ? offs[3 * k + i] : 0);
    for (int j = 0; j < 3; ++j)
        pl[j] = (R)rm[0 + j] * w[0] + (R)rm[3 + j] * w[1] + (R)rm[6 + j] * w[2];
}

void FN(or_navigate_safety)(int mother_kind, const double *mother_par, int nd,
                            const int32_t *kinds, const double *pars, const double *rots,
                            const double *trs, const double *offsets, int64_t n,
                            const double *x, const double *y, const double *z, double *safety)
{
    FN(vol) v = { mother_kind, mother_par, nd, kinds, pars, rots, trs };
    R offs[3 * OR_MAX_DAUGHTERS];
    if (offsets)
        for (int i = 0; i < 3 * nd; ++i) offs[i] = offsets[i];
    for (int64_t i = 0; i < n; ++i) {
        R p[3] = { x[i], y[i], z[i] };
        R best = FN(safety)(mother_kind, mother_par, p[0], p[1], p[2]);
        for (int k = 0; k < nd; ++k) {
            R pl[3];
            FN(local_point)(&v, k, p, offsets ? offs : 0, pl);
            R s = FN(safety)(kinds[k], pars + OR_NPAR * k, pl[0], pl[1], pl[2]);
            if (s < best) best = s;
        }
        safety[i] = (double)best;
    }
}

void FN(or_locate)(int mother_kind, const double *mother_par, int nd, const int32_t *kinds,
                   const double *pars, const double *rots, const double *trs,
                   const double *offsets, int64_t n, const double *x, const double *y,
                   const double *z, int32_t *where)
{
    FN(vol) v = { mother_kind, mother_par, nd, kinds, pars, rots, trs };
    R offs[3 * OR_MAX_DAUGHTERS];
    if (offsets)
        for (int i = 0; i < 3 * nd; ++i) offs[i] = offsets[i];
    for (int64_t i = 0; i < n; ++i) {
        R p[3] = { x[i], y[i], z[i] };
        int32_t w = -2;
        if (FN(contains)(mother_kind, mother_par, p[0], p[1], p[2])) {
            w = -1;
            for (int k = 0; k < nd && w < 0; ++k) {
                R pl[3];
                FN(local_point)(&v, k, p, offsets ? offs : 0, pl);
                if (FN(contains)(kinds[k], pars + OR_NPAR * k, pl[0], pl[1], pl[2])) w = k;
            }
        }
        where[i] = w;
    }
}

/*
 * geonav — basket-wide geometry queries and the simple vector navigator on
 * AMD MI355X (gfx950), after "Vectorising the detector geometry to optimize
 * particle transport" (Apostolakis, Brun, Carminati, Gheata, Wenzel).
 *
 * C ABI of libgeonav.so. All functions return an int status (GEO_OK or a
 * negative GEO_ERR_*); no C++ exception crosses this boundary. Computation is
 * FP64 throughout.
 *
 * Memory and ownership
 *   - Track arrays and output arrays are DEVICE pointers owned by the caller,
 *     8-byte aligned (4 for int32 outputs, 1 for uint8), not aliasing each
 *     other. Every call is asynchronous on the given stream; the caller keeps
 *     the buffers alive until the stream has passed the call.
 *   - Descriptor structs (geo_shape, geo_volume_desc, geo_basket arrays) are
 *     HOST memory, read during the call only.
 *   - A geo_geometry handle owns device copies of its volumes.
 *
 * Conventions (section 3.1 names the shapes and queries; the parameter
 * conventions below follow ROOT-style half-lengths, centred on the origin,
 * z as the symmetry axis):
 *   GEO_BOX  par = {dx, dy, dz}                          |x|<=dx, |y|<=dy, |z|<=dz
 *   GEO_TUBE par = {rmin, rmax, dz}                      rmin<=r<=rmax, |z|<=dz
 *   GEO_CONE par = {dz, rmin1, rmax1, rmin2, rmax2}      radii "1" at z=-dz and
 *            "2" at z=+dz, varying linearly in z
 *   GEO_TUBS par = {rmin, rmax, dz, phi1, dphi}          the tube and cone cut to
 *   GEO_CONS par = {dz, rmin1, rmax1, rmin2, rmax2, phi1, dphi}   the azimuths
 *            [phi1, phi1 + dphi] (radians, 0 < dphi <= 2 pi), z axis included
 *            (section 3.1 names the segmented forms of tube and cone); two
 *            flat faces close the cut. dphi = 2 pi is the uncut base solid.
 *   GEO_PCON par = {phi1, dphi, nz, z_0, rmin_0, rmax_0, ..., z_{nz-1},
 *            rmin_{nz-1}, rmax_{nz-1}}   the polycone (section 3.1: a sequence
 *            of connected cone and tube sections, "few z segments"): nz planes,
 *            2 <= nz <= GEO_PCON_MAX_PLANES (an integral value), z strictly
 *            increasing, 0 <= rmin <= rmax at each plane; between consecutive
 *            planes both radii vary linearly in z. Cut to [phi1, phi1 + dphi]
 *            like the segments (dphi = 2 pi: uncut).
 *   Parameters beyond those a kind reads are ignored.
 *   Shapes are closed sets. Directions are not renormalised: distances are
 *   the ray parameter t of p + t*d (the length when |d| = 1). Every
 *   finite t must stay below GEO_BIG, the value of a miss, so |d| is at
 *   least 1e-30 times the largest extent of the geometry; and |d| is at
 *   most 1e100 (the ray-surface quadratics square products of |d| with
 *   coordinates and section slopes: at |d| near 1e150 a steep polycone
 *   section far from the track overflows them). Outside that range the
 *   results are not specified.
 *   A line that never reaches the boundary gives GEO_BIG.
 */
#ifndef GEONAV_H
#define GEONAV_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GEO_BIG 1e30
#define GEO_MAX_DAUGHTERS 1024
#define GEO_CENSUS_SLOTS 16
#define GEO_PCON_MAX_PLANES 8
#define GEO_NPAR (3 + 3 * GEO_PCON_MAX_PLANES) /* parameters per shape */

enum { GEO_BOX = 0, GEO_TUBE = 1, GEO_CONE = 2, GEO_TUBS = 3, GEO_CONS = 4, GEO_PCON = 5 };

/* Queries of section 3.1: inside/outside check, minimum distance to any
 * boundary, distance along the line of flight to leave / to enter. */
enum { GEO_CONTAINS = 0, GEO_SAFETY = 1, GEO_DIST_IN = 2, GEO_DIST_OUT = 3 };

enum {
    GEO_OK = 0,
    GEO_ERR_INVALID_ARG = -1, /* bad pointer, size, kind, query, volume, shape or alignment */
    GEO_ERR_HIP = -2,         /* a HIP runtime call failed; geo_strerror gives its message */
    GEO_ERR_NOMEM = -3        /* a device or pinned host allocation failed */
};

/* A basket (section 2): the tracks of one logical volume as six SoA device
 * arrays of length n (origin x, y, z and direction ux, uy, uz). */
typedef struct {
    const double *x, *y, *z, *ux, *uy, *uz;
    int64_t n;
} geo_tracks;

typedef struct {
    int32_t kind; /* GEO_BOX, GEO_TUBE, GEO_CONE, GEO_TUBS, GEO_CONS or GEO_PCON */
    int32_t _pad;
    double par[GEO_NPAR];
} geo_shape;

/* Placement of a daughter in its mother (the coordinate transformations of
 * section 3.1): a daughter-frame point q is at rot * q + tr in the mother
 * frame. rot is row-major and must be a proper rotation (orthonormal to
 * 1e-12, determinant +1). */
typedef struct {
    double rot[9];
    double tr[3];
} geo_placement;

/* A logical volume (Fig. 1): a mother shape and its placed daughters. */
typedef struct {
    geo_shape mother;
    int32_t ndaughters; /* 0 .. GEO_MAX_DAUGHTERS */
    int32_t _pad;
    const geo_shape *daughters;      /* host, ndaughters */
    const geo_placement *placements; /* host, ndaughters */
} geo_volume_desc;

/* A basket of the batched call: n tracks of volume `volume` starting at
 * `offset` in the shared track pool. */
typedef struct {
    int32_t volume;
    int32_t _pad;
    int64_t offset;
    int64_t n;
} geo_basket;

typedef struct geo_geometry geo_geometry;

/* Copy nvol volumes to the current device and return a handle.
 * Validation: kinds known, parameters finite, box half-lengths > 0,
 * 0 <= rmin <= rmax with rmax > 0 (cone: at both ends, rmax1 + rmax2 > 0),
 * dz > 0, segments and polycones 0 < dphi <= 2 pi, polycone planes as
 * above (each section with rmax > 0 at one of its planes at least),
 * rotations proper to 1e-12. A tube or tube-segment daughter is held as
 * the equal-radii cone (segment), the same solid, and evaluated by the
 * cone's code in the navigators. Errors: GEO_ERR_INVALID_ARG,
 * GEO_ERR_NOMEM, GEO_ERR_HIP; *out is NULL on error. */
int geo_geometry_create(const geo_volume_desc *volumes, int32_t nvol, geo_geometry **out);

/* Release the handle and its device memory. Synchronises the device first.
 * NULL is a no-op. */
int geo_geometry_destroy(geo_geometry *g);

/* Shape queries of section 3.1 over a whole basket: one launch evaluates
 * `query` for the shape `s` (host struct, in its own frame) at every track.
 * out: uint8_t[n] (GEO_CONTAINS: 1 inside, 0 outside) or double[n]
 * (GEO_SAFETY: Euclidean distance to the surface; GEO_DIST_IN: distance to
 * leave, 0 for a point outside; GEO_DIST_OUT: distance to enter, 0 for a
 * point inside). Contains and Safety ignore ux, uy, uz (they may be NULL).
 * n == 0 is a no-op. */
int geo_shape_query(const geo_shape *s, int32_t query, geo_tracks t, void *out, hipStream_t stream);

/* The simple navigator of section 3 (Fig. 1b) over one basket of `volume`:
 *   step[i] = min( DistFromInside_mother(p_i, d_i),
 *                  min_k DistFromOutside_k(R_k^T (p_i - T_k - delta_k), R_k^T d_i) )
 *   hit[i]  = -1 if the mother attains it, else the daughter index k;
 *            ties go to the mother, then to the lowest k.
 * offsets: device double[ndaughters * 3] (delta_k, x/y/z per daughter) or
 * NULL for zero. hitpt: device double[3 * n] (SoA rows x, y, z of
 * p + step * d) or NULL. Tracks should start inside the mother and outside
 * every daughter (section 3.2's benchmark protocol); a track inside daughter
 * k gets step 0 (hit = the first such k), a track outside the mother gets
 * step 0 and hit -1. */
int geo_navigate_basket(const geo_geometry *g, int32_t volume, geo_tracks t, const double *offsets,
                        double *step, int32_t *hit, double *hitpt, hipStream_t stream);

/* The navigator's isotropic safety (section 3: safe distances to the
 * volume's boundaries) for every point of a basket of `volume`:
 *   safety[i] = min( Safety_mother(p_i), min_k Safety_k(R_k^T (p_i - T_k - delta_k)) )
 * with each Safety the Euclidean distance to that shape's surface, so for a
 * point in the mother's own part it is the distance to the nearest boundary
 * of the volume. Only x, y, z of t are read (directions may be NULL).
 * offsets as for geo_navigate_basket. safety: device double[n]. */
int geo_navigate_safety(const geo_geometry *g, int32_t volume, geo_tracks t, const double *offsets,
                        double *safety, hipStream_t stream);

/* Localization (section 3: the containing volume of a point): where[i] = the
 * lowest daughter index k whose shape contains R_k^T (p_i - T_k - delta_k),
 * -1 for a point in the mother but in no daughter, -2 for a point outside
 * the mother. Only x, y, z of t are read. where: device int32[n]. */
int geo_locate(const geo_geometry *g, int32_t volume, geo_tracks t, const double *offsets, int32_t *where,
               hipStream_t stream);

/* Many baskets of possibly different volumes in ONE navigator launch,
 * after a small kernel that expands the baskets into tiles (the two as two
 * launches on the stream, or as a replay of a cached HIP graph: see
 * geo_set_batched_graph). baskets: host array of nb entries
 * indexing into the shared pool `all`; step and hit are indexed like the
 * pool (entry offset + j for track j of a basket); pool entries not covered
 * by any basket are left untouched. Results are bit-identical to
 * geo_navigate_basket on each basket with offsets = NULL. Baskets of one
 * volume given one after another whose tracks follow one another in the
 * pool are navigated as one (their tiles fill whole wavefronts across the
 * basket boundaries); that changes no output.
 * The handle keeps per-call state (tile buffer, graph, a ring of pinned
 * staging buffers): calls on one handle must come from one host thread at a
 * time and be ordered on the device (the same stream, or streams the caller
 * synchronises); a call may return before the device has run it. */
int geo_navigate_batched(geo_geometry *g, const geo_basket *baskets, int32_t nb, geo_tracks all,
                         double *step, int32_t *hit, hipStream_t stream);

/* Adjoint of the navigator for one basket (recomputes the forward pass, then
 * differentiates the surface that determined each step, by the implicit-
 * function theorem on that surface). With upstream gradients gstep (double[n]
 * or NULL = 0) for the step and ghit (double[3 * n] SoA or NULL = 0) for the
 * hit point h = p + step * d, it writes
 *   g_o   (double[3 * n] SoA, or NULL to skip): d/dp of sum_i gstep_i s_i + ghit_i . h_i
 *   g_d   (double[3 * n] SoA, or NULL to skip): d/dd of the same
 *   g_off (double[ndaughters * 3], or NULL to skip): d/d delta_k summed over
 *         the basket; overwritten, deterministic (fixed reduction order).
 * Tracks whose step is 0 (outside the mother or inside a daughter) or that
 * never reach a boundary contribute 0. At a non-smooth point (an edge, a tie
 * between volumes) the gradient of the surface the forward pass picked is
 * used. With offsets and culling, a small kernel first writes the volume's
 * culling records moved by the offsets into a buffer of the handle, which
 * the forward pass's culling tests read. Calls on one handle share that
 * buffer and a partial-sum buffer: they must be stream-ordered (no
 * concurrent backward calls on one handle). */
int geo_navigate_backward(const geo_geometry *g, int32_t volume, geo_tracks t, const double *offsets,
                          const double *gstep, const double *ghit, double *g_o, double *g_d,
                          double *g_off, hipStream_t stream);

/* geo_navigate_backward for callers that cannot allocate memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid it): the
 * same arguments and results (bit for bit), but the partial sums of the
 * offset gradient live in a static device buffer of the library (3 MiB, one
 * per GPU, held until the process ends) instead of the handle's, the
 * culling tests apply the offsets themselves (no shifted records are
 * written into the handle), and the call allocates nothing. The buffer holds 2048 * 3 * 64 doubles: any
 * track count with up to 64 daughters; with more, a call whose partial sums
 * (min(ceil(n / 256), 2048) rows of 3 * ndaughters) do not fit fails with
 * GEO_ERR_INVALID_ARG before launching anything. Every call on one GPU shares
 * that GPU's buffer (nothing in it needs to start at zero): calls that
 * overlap on one GPU (concurrent streams, host threads) race; order them. */
int geo_navigate_backward_noalloc(const geo_geometry *g, int32_t volume, geo_tracks t, const double *offsets,
                                  const double *gstep, const double *ghit, double *g_o, double *g_d,
                                  double *g_off, hipStream_t stream);

/* Instrumented run of geo_navigate_batched (same outputs, not for timing):
 * launches directly (no graph) a variant of the batched kernel that tallies
 * the work it does. counts (host uint64_t[GEO_CENSUS_SLOTS]):
 *   counts[2 * kind + hole]  lane-evaluations of DistFromOutside for daughters
 *                            of that kind (kind 0..4 as above, 5 an uncut
 *                            polycone, 6 a cut one; hole = 1 for a shape with
 *                            an inner surface): with culling, one per
 *                            (track, daughter) pair that passed the culling
 *                            test; without, every active lane of a
 *                            wavefront that evaluates the daughter,
 *   counts[14]               lane culling tests (0 with culling off),
 *   counts[15]               tracks navigated (mother DistFromInside).
 * Synchronises the stream. */
int geo_navigate_batched_census(geo_geometry *g, const geo_basket *baskets, int32_t nb, geo_tracks all,
                                double *step, int32_t *hit, uint64_t counts[GEO_CENSUS_SLOTS],
                                hipStream_t stream);

/* Time the candidate launch shapes of the batched kernel (tracks per lane
 * 1/2/4/8 x waves per SIMD 0/2/3/4/6/8) on these baskets, as bursts of
 * back-to-back calls after a warm-up, then, at the fastest shape, the two
 * kernels as a graph replay against two launches; keep the fastest in the
 * handle; also records it in the JSON cache named by the
 * GEONAV_AUTOTUNE_CACHE environment variable, if set. Writes step/hit
 * scratch internally; synchronises the stream. */
int geo_autotune(geo_geometry *g, const geo_basket *baskets, int32_t nb, geo_tracks all,
                 hipStream_t stream);

/* Launch shape of the batched kernel. tracks_per_lane (1, 2, 4 or 8) sets the
 * tile size (64 * tracks_per_lane tracks of one volume per wavefront task);
 * waves_per_simd 1..8 selects the persistent kernel with that many
 * wavefronts per SIMD pulling tiles from per-XCD queues, 0 selects one
 * wavefront per tile scheduled by the hardware. Default 4 and 0; the
 * autotuner may change them. Results do not depend on the launch shape. */
int geo_get_launch_config(const geo_geometry *g, int32_t *tracks_per_lane, int32_t *waves_per_simd);
int geo_set_launch_config(geo_geometry *g, int32_t tracks_per_lane, int32_t waves_per_simd);

/* How geo_navigate_batched submits its two kernels: use_graph = 1 replays a
 * HIP graph built on the first call (its kernel arguments updated in place
 * on later calls), 0 launches them one after the other on the stream. The
 * default is 0 (on an MI355X the replay measured about 6 us more per call);
 * the autotuner may change it. Results do not depend on it. GEO_ERR_INVALID_ARG
 * for a NULL handle or pointer, or use_graph other than 0 or 1. */
int geo_get_batched_graph(const geo_geometry *g, int32_t *use_graph);
int geo_set_batched_graph(geo_geometry *g, int32_t use_graph);

/* Culling in the navigators (basket, batched, backward): a daughter is not
 * evaluated for a track whose line cannot enter the daughter's bounding
 * sphere (radius enlarged by 1e-6 relative + 1e-6) before the mother's exit.
 * The (track, daughter) pairs that pass are queued in LDS and evaluated one
 * pair per lane. A culled daughter could neither lower a step nor
 * win a tie, so results are bit-identical with culling on or off; only the
 * work done changes. Applies likewise to geo_navigate_safety (a daughter
 * whose sphere is farther than the mother's safety) and geo_locate (a point
 * outside the sphere). On by default. */
int geo_set_culling(geo_geometry *g, int32_t enable);
int geo_get_culling(const geo_geometry *g, int32_t *enabled);

/* Timing of the batched navigator kernel alone, for measurement. With
 * enable != 0, the graph of geo_navigate_batched records two events of its
 * own, just before and just after the navigator kernel (the tile expansion
 * before it is outside the interval); geo_batched_kernel_ms then waits for
 * the most recent such call to finish and returns that kernel's duration in
 * milliseconds. Enabling creates the two events (GEO_ERR_HIP if that
 * fails); the graph is rebuilt on the next call. Results do not change.
 * geo_batched_kernel_ms fails with GEO_ERR_INVALID_ARG when timing is off or
 * no batched call has run since it was enabled. */
int geo_set_kernel_timing(geo_geometry *g, int32_t enable);
int geo_batched_kernel_ms(geo_geometry *g, float *ms);

/* Message for a status code; for the most recent failure on the calling
 * thread it includes that failure's detail. Never NULL. */
const char *geo_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* GEONAV_H */

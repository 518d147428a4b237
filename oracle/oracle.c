/*
 * CPU oracle for the basket shape queries and the simple navigator of
 * "Vectorising the detector geometry to optimize particle transport"
 * (section 3, Fig. 1, and section 3.1): box, tube, cone, the segmented
 * tube and cone, and the polycone with few z sections.
 *
 * TEST INFRASTRUCTURE. Only the test-suite, the smoke check and the CPU
 * baseline of the benchmark load this library; the product path (the HIP
 * library) never calls it and shares no code, header or table with it.
 *
 * Each query is its plain definition, computed by an algorithm different
 * from the GPU path (intervals of the flight line rather than per-surface
 * candidates):
 *   Contains         closed-set membership;
 *   Safety           Euclidean distance to the boundary (box: per-face /
 *                    per-axis excess; tube and cone: planar distance to the
 *                    edges of the (r, z) profile);
 *   DistFromOutside  smallest t >= 0 with p + t d in the shape, 0 if p is
 *                    inside, OR_BIG if the line never enters;
 *   DistFromInside   upper end of the line interval holding t = 0, 0 if p
 *                    is outside;
 *   navigator        Fig. 1: min of the mother's DistFromInside and every
 *                    daughter's DistFromOutside in the daughter's frame;
 *   adjoint          central finite differences of the navigator.
 *
 * Every function is built twice from oracle_body.h: in double (suffix _d)
 * and in x87 long double (suffix _ld). The long-double build is the
 * higher-precision rerun used to flag ill-conditioned tracks.
 * Compiled with -O2 -ffp-contract=off (no fused multiply-add, no fast-math).
 */
#include <math.h>
#include <stdint.h>
#include <tgmath.h>

#define OR_BOX 0
#define OR_TUBE 1
#define OR_CONE 2
#define OR_TUBS 3
#define OR_CONS 4
#define OR_PCON 5

#define OR_CONTAINS 0
#define OR_SAFETY 1
#define OR_DIST_IN 2
#define OR_DIST_OUT 3

#define OR_BIG 1e30
#define OR_PCON_MAX 8            /* z planes of a polycone */
#define OR_NPAR (3 + 3 * OR_PCON_MAX)   /* parameters per shape */
#define OR_MAX_DAUGHTERS 1024
#define OR_MAX_IVAL (5 * OR_PCON_MAX)   /* line intervals of one shape */
#define OR_TWO_PI 6.283185307179586476925286766559005768L
#define OR_FULL_TURN ((double)OR_TWO_PI)   /* dphi at or above: uncut */

#define R double
#define FN(n) n##_d
#include "oracle_body.h"
#undef R
#undef FN

#define R long double
#define FN(n) n##_ld
#include "oracle_body.h"
#undef R
#undef FN

int or_max_daughters(void) { return OR_MAX_DAUGHTERS; }

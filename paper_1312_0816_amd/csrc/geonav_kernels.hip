// Kernels of libgeonav for gfx950 and their launchers.
//
//  k_shape_query     one query of one shape over a basket (section 3.1);
//                    streaming, one lane per track, HBM-bound (the polycone
//                    and the cone segment's Safety are ALU-bound).
//  k_nav_basket      the simple navigator (section 3, Fig. 1b) over one
//                    basket: culling tests in lockstep queue (track, daughter)
//                    pairs in LDS, evaluated one pair per lane; bound by VALU
//                    issue (with culling off, every lane walks every daughter).
//  k_nav_safety      the navigator's isotropic safety (section 3) per point;
//  k_nav_locate      the daughter holding each point (localization);
//  k_build_tiles     expands a host-sorted basket list into tiles of at most
//                    64 x U tracks of one volume (largest cost first);
//  k_nav_tiles       the per-track navigator over all tiles of many baskets
//                    of many volumes in one launch, one wavefront per tile;
//  k_nav_persistent  the same with a machine-sized grid whose wavefronts
//                    pull tiles from per-XCD queues;
//  k_shift_cull      a volume's culling records moved by the daughter offsets
//                    of one adjoint call;
//  k_nav_backward    adjoint of the navigator (recompute + implicit-function
//                    gradient of the surface that set the step) with
//                    per-workgroup partial sums of the offset gradient;
//  k_reduce_partials fixed-order reduction of those partials.
#include <mutex>

#include "geonav_internal.hpp"

namespace gn {

// Runs STMT with the compile-time constant KS set to the runtime kind set.
#define GN_KSET(kset, STMT)                                 \
    do {                                                    \
        if ((kset) == kSetBasic) {                          \
            constexpr int KS = kSetBasic;                   \
            STMT;                                           \
        } else if ((kset) == kSetSeg) {                     \
            constexpr int KS = kSetSeg;                     \
            STMT;                                           \
        } else {                                            \
            constexpr int KS = kSetAll;                     \
            STMT;                                           \
        }                                                   \
    } while (0)

// ------------------------------------------------------------ shape queries
// A polycone's sections come by value with the arguments (`pc`, unused for
// the other kinds).
template <int KIND, int Q>
__global__ __launch_bounds__(kBlock) void k_shape_query(ShapeRec s, PconRec pc, TracksDev t,
                                                        void *out) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= t.n) return;
    const double x = t.x[i], y = t.y[i], z = t.z[i];
    if (Q == 0) {
        static_cast<uint8_t *>(out)[i] = shape_contains<KIND>(s, &pc, x, y, z) ? 1 : 0;
        return;
    }
    double r;
    if (Q == 1) {
        r = shape_safety<KIND>(s, &pc, x, y, z);
    } else {
        const double ux = t.ux[i], uy = t.uy[i], uz = t.uz[i];
        int sid;
        if (Q == 2) r = shape_dist_in<KIND>(s, &pc, x, y, z, ux, uy, uz, sid);
        else r = shape_dist_out<KIND>(s, &pc, x, y, z, ux, uy, uz, sid);
    }
    static_cast<double *>(out)[i] = r;
}

template <int KIND>
static hipError_t launch_shape_kind(const ShapeRec &s, const PconRec &pc, int query,
                                    const TracksDev &t, void *out, hipStream_t st) {
    const dim3 grid((unsigned)((t.n + kBlock - 1) / kBlock)), block(kBlock);
    switch (query) {
        case 0: hipLaunchKernelGGL((k_shape_query<KIND, 0>), grid, block, 0, st, s, pc, t, out); break;
        case 1: hipLaunchKernelGGL((k_shape_query<KIND, 1>), grid, block, 0, st, s, pc, t, out); break;
        case 2: hipLaunchKernelGGL((k_shape_query<KIND, 2>), grid, block, 0, st, s, pc, t, out); break;
        default: hipLaunchKernelGGL((k_shape_query<KIND, 3>), grid, block, 0, st, s, pc, t, out); break;
    }
    return hipGetLastError();
}

hipError_t launch_shape_query(const ShapeRec &s, const PconRec &pc, int query, const TracksDev &t,
                              void *out, hipStream_t st) {
    if (t.n == 0) return hipSuccess;
    switch (s.kind) {
        case kBox: return launch_shape_kind<kBox>(s, pc, query, t, out, st);
        case kTube: return launch_shape_kind<kTube>(s, pc, query, t, out, st);
        case kCone: return launch_shape_kind<kCone>(s, pc, query, t, out, st);
        case kTubs: return launch_shape_kind<kTubs>(s, pc, query, t, out, st);
        case kCons: return launch_shape_kind<kCons>(s, pc, query, t, out, st);
        case kPcon: return launch_shape_kind<kPcon>(s, pc, query, t, out, st);
        default: return launch_shape_kind<kPcons>(s, pc, query, t, out, st);
    }
}

// ---------------------------------------------------------- basket navigator
// With culling, one wavefront takes U rounds of 64 tracks (compacted
// evaluation; more tracks per wavefront fill more lanes of each batch of
// queued pairs).
// Volumes holding every kind: the polycone's code would take the kernel to
// 102 VGPRs, 4 wavefronts per SIMD; held to 96 (5 wavefronts, a few bytes
// spilled to scratch) the mixed detector's navigator runs 7 % faster.
template <bool HAS_OFFS, bool HITPT, bool CULL, int KSET, int U = 1>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(KSET == kSetAll ? 5 : 1))) void k_nav_basket(const VolumeRec *__restrict__ vol,
                                                       const DaughterRec *__restrict__ dau,
                                                       const CullRec *__restrict__ cul,
                                                       TracksDev t, const double *__restrict__ offs,
                                                       double *__restrict__ step,
                                                       int32_t *__restrict__ hit,
                                                       double *__restrict__ hitpt) {
    if constexpr (CULL && KSET != kSetBasic) {
        // volumes of more kinds: the workgroup's wavefronts pool their last
        // flush (a wavefront past the basket's end takes part with no tracks)
        __shared__ NavScratch<U> scr[kBlock / 64];
        __shared__ PoolInfo<kBlock / 64> pool;
        const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // (uniform)
        const int64_t base = ((int64_t)blockIdx.x * (kBlock / 64) + wave) * 64 * U;
        const int64_t left = t.n - base;
        const int count = left <= 0 ? 0 : (left < 64 * U ? (int)left : 64 * U);
        nav_compact_pooled<U, kBlock / 64, HAS_OFFS, HITPT, KSET>(*vol, dau, cul, 0, offs, t, base, count, scr,
                                                                  pool, true, wave, (int)(threadIdx.x & 63),
                                                                  step, hit, hitpt);
        return;
    }
    if constexpr (CULL) {
        // (box, tube and cone only: pooling gains nothing measurable)
        __shared__ NavScratch<U> scr[kBlock / 64];
        const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // (uniform)
        const int64_t base = ((int64_t)blockIdx.x * (kBlock / 64) + wave) * 64 * U;
        if (base >= t.n) return;
        const int count = t.n - base < 64 * U ? (int)(t.n - base) : 64 * U;
        nav_compact<U, HAS_OFFS, HITPT, false, KSET>(*vol, dau, cul, offs, t, base, count, scr[wave],
                                                     (int)(threadIdx.x & 63), step, hit, hitpt);
        return;
    }
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= t.n) return;
    const double x = t.x[i], y = t.y[i], z = t.z[i];
    const double ux = t.ux[i], uy = t.uy[i], uz = t.uz[i];
    double best;
    int h, sid;
    nav_track<HAS_OFFS, false, false, KSET>(*vol, dau, cul, offs, x, y, z, ux, uy, uz, best, h, sid);
    step[i] = best;
    hit[i] = h;
    if (HITPT) {
        const int64_t n = t.n;
        hitpt[i] = fma(best, ux, x);
        hitpt[n + i] = fma(best, uy, y);
        hitpt[2 * n + i] = fma(best, uz, z);
    }
}

template <bool CULL, int KSET, int U = 1>
static void launch_basket_variant(dim3 grid, const VolumeRec *vol, const DaughterRec *dau,
                                  const CullRec *cul, const TracksDev &t, const double *offs, double *step, int32_t *hit,
                                  double *hitpt, hipStream_t st) {
    const dim3 block(kBlock);
    if (offs) {
        if (hitpt) hipLaunchKernelGGL((k_nav_basket<true, true, CULL, KSET, U>), grid, block, 0, st, vol, dau, cul, t, offs, step, hit, hitpt);
        else hipLaunchKernelGGL((k_nav_basket<true, false, CULL, KSET, U>), grid, block, 0, st, vol, dau, cul, t, offs, step, hit, hitpt);
    } else {
        if (hitpt) hipLaunchKernelGGL((k_nav_basket<false, true, CULL, KSET, U>), grid, block, 0, st, vol, dau, cul, t, offs, step, hit, hitpt);
        else hipLaunchKernelGGL((k_nav_basket<false, false, CULL, KSET, U>), grid, block, 0, st, vol, dau, cul, t, offs, step, hit, hitpt);
    }
}

// Baskets of at least kBasketWide tracks run 4 rounds per wavefront (still
// about 4096 wavefronts, several per SIMD); smaller baskets one round. (8
// rounds when the volume holds every kind, which fills each batch of queued
// pairs better, gave 5 % with the running minima in LDS alone; with the
// track cache beside them its LDS allows 3 wavefronts per SIMD instead of
// 5: 162 against 141 us on a 2^22-track basket of the mixed detector.)
constexpr int64_t kBasketWide = (int64_t)1 << 20;

hipError_t launch_nav_basket(const VolumeRec *vol, const DaughterRec *dau, const CullRec *cul,
                             const TracksDev &t, const double *offs, double *step, int32_t *hit,
                             double *hitpt, bool cull, int kset, hipStream_t st) {
    if (t.n == 0) return hipSuccess;
    const dim3 grid((unsigned)((t.n + kBlock - 1) / kBlock));
    if (cull && t.n >= kBasketWide) {
        const dim3 grid4((unsigned)((t.n + 4 * kBlock - 1) / (4 * kBlock)));
        GN_KSET(kset, (launch_basket_variant<true, KS, 4>(grid4, vol, dau, cul, t, offs, step, hit, hitpt, st)));
    } else if (cull) {
        GN_KSET(kset, (launch_basket_variant<true, KS>(grid, vol, dau, cul, t, offs, step, hit, hitpt, st)));
    } else {
        GN_KSET(kset, (launch_basket_variant<false, KS>(grid, vol, dau, cul, t, offs, step, hit, hitpt, st)));
    }
    return hipGetLastError();
}

// -------------------------------------------------- safety and locate
template <bool HAS_OFFS, bool CULL, int KSET, int U = 1>
__global__ __launch_bounds__(kBlock) void k_nav_safety(const VolumeRec *__restrict__ vol,
                                                       const DaughterRec *__restrict__ dau,
                                                       const CullRec *__restrict__ cul, TracksDev t,
                                                       const double *__restrict__ offs,
                                                       double *__restrict__ out) {
    if constexpr (CULL) {
        __shared__ PointScratch<U> scr[kBlock / 64];
        const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // (uniform)
        const int64_t base = ((int64_t)blockIdx.x * (kBlock / 64) + wave) * 64 * U;
        if (base >= t.n) return;
        const int count = t.n - base < 64 * U ? (int)(t.n - base) : 64 * U;
        point_compact<0, HAS_OFFS, KSET, U>(*vol, dau, cul, offs, t, base, count, scr[wave],
                                            (int)(threadIdx.x & 63), out, nullptr);
        return;
    }
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= t.n) return;
    out[i] = nav_safety<HAS_OFFS, KSET>(*vol, dau, cul, offs, t.x[i], t.y[i], t.z[i]);
}

template <bool HAS_OFFS, bool CULL, int KSET, int U = 1>
__global__ __launch_bounds__(kBlock) void k_nav_locate(const VolumeRec *__restrict__ vol,
                                                       const DaughterRec *__restrict__ dau,
                                                       const CullRec *__restrict__ cul, TracksDev t,
                                                       const double *__restrict__ offs,
                                                       int32_t *__restrict__ out) {
    if constexpr (CULL) {
        __shared__ PointScratch<U> scr[kBlock / 64];
        const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // (uniform)
        const int64_t base = ((int64_t)blockIdx.x * (kBlock / 64) + wave) * 64 * U;
        if (base >= t.n) return;
        const int count = t.n - base < 64 * U ? (int)(t.n - base) : 64 * U;
        point_compact<1, HAS_OFFS, KSET, U>(*vol, dau, cul, offs, t, base, count, scr[wave],
                                            (int)(threadIdx.x & 63), nullptr, out);
        return;
    }
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= t.n) return;
    out[i] = nav_locate<HAS_OFFS, KSET>(*vol, dau, cul, offs, t.x[i], t.y[i], t.z[i]);
}

template <bool CULL, int KSET, int U = 1>
static void launch_safety_variant(dim3 grid, const VolumeRec *vol, const DaughterRec *dau,
                                  const CullRec *cul, const TracksDev &t, const double *offs,
                                  double *out, hipStream_t st) {
    if (offs) hipLaunchKernelGGL((k_nav_safety<true, CULL, KSET, U>), grid, dim3(kBlock), 0, st, vol, dau, cul, t, offs, out);
    else hipLaunchKernelGGL((k_nav_safety<false, CULL, KSET, U>), grid, dim3(kBlock), 0, st, vol, dau, cul, t, offs, out);
}

template <bool CULL, int KSET, int U = 1>
static void launch_locate_variant(dim3 grid, const VolumeRec *vol, const DaughterRec *dau,
                                  const CullRec *cul, const TracksDev &t, const double *offs,
                                  int32_t *out, hipStream_t st) {
    if (offs) hipLaunchKernelGGL((k_nav_locate<true, CULL, KSET, U>), grid, dim3(kBlock), 0, st, vol, dau, cul, t, offs, out);
    else hipLaunchKernelGGL((k_nav_locate<false, CULL, KSET, U>), grid, dim3(kBlock), 0, st, vol, dau, cul, t, offs, out);
}

// One round of 64 points per wavefront: with four (as the basket navigator
// takes for large baskets) both ran 5-15 % slower on the toy detector.
hipError_t launch_nav_safety(const VolumeRec *vol, const DaughterRec *dau, const CullRec *cul,
                             const TracksDev &t, const double *offs, double *out, bool cull,
                             int kset, hipStream_t st) {
    if (t.n == 0) return hipSuccess;
    const dim3 grid((unsigned)((t.n + kBlock - 1) / kBlock));
    if (cull) GN_KSET(kset, (launch_safety_variant<true, KS>(grid, vol, dau, cul, t, offs, out, st)));
    else GN_KSET(kset, (launch_safety_variant<false, KS>(grid, vol, dau, cul, t, offs, out, st)));
    return hipGetLastError();
}

hipError_t launch_nav_locate(const VolumeRec *vol, const DaughterRec *dau, const CullRec *cul,
                             const TracksDev &t, const double *offs, int32_t *out, bool cull,
                             int kset, hipStream_t st) {
    if (t.n == 0) return hipSuccess;
    const dim3 grid((unsigned)((t.n + kBlock - 1) / kBlock));
    if (cull) GN_KSET(kset, (launch_locate_variant<true, KS>(grid, vol, dau, cul, t, offs, out, st)));
    else GN_KSET(kset, (launch_locate_variant<false, KS>(grid, vol, dau, cul, t, offs, out, st)));
    return hipGetLastError();
}

// ------------------------------------------------------------------ batched
// A tile holds at most 64 * U tracks of one volume: U rounds of one track
// per lane, so the volume and its daughters are uniform over the wavefront.
// Tiles come in order of decreasing per-track cost (the host sorts the
// baskets by daughter count; k_build_tiles expands them in that order).
template <int U, bool CULL, bool COUNT, int KSET>
__device__ __forceinline__ void run_tile(const Tile &tl, const VolumeRec *__restrict__ vols,
                                         const DaughterRec *__restrict__ dau_all,
                                         const CullRec *__restrict__ cul_all, const TracksDev &t,
                                         double *__restrict__ step, int32_t *__restrict__ hit,
                                         unsigned long long *census, int lane,
                                         NavScratch<U> *scr) {
    const VolumeRec &v = vols[tl.volume];
    const DaughterRec *dau = dau_all + v.first;
    const CullRec *cul = cul_all + v.first;
    if constexpr (CULL) {
        nav_compact<U, false, false, COUNT, KSET>(v, dau, cul, nullptr, t, tl.offset, tl.count, *scr,
                                                  lane, step, hit, nullptr, census);
        return;
    }
#pragma unroll 1
    for (int u = 0; u < U; ++u) {
        const int j = u * 64 + lane;
        if (j < tl.count) {
            const int64_t i = tl.offset + j;
            const double x = t.x[i], y = t.y[i], z = t.z[i];
            const double ux = t.ux[i], uy = t.uy[i], uz = t.uz[i];
            double best;
            int h, sid;
            nav_track<false, false, COUNT, KSET>(v, dau, cul, nullptr, x, y, z, ux, uy, uz,
                                                       best, h, sid, census);
            step[i] = best;
            hit[i] = h;
        }
    }
}

// Persistent form: a grid sized to the machine; tiles are dealt round-robin
// into kQueues queues (tile i to queue i mod kQueues, in order), each with its
// own cursor on its own 256-byte line, so the atomics that hand out tiles
// spread over kQueues addresses instead of contending on one. A wavefront
// drains the queue of its workgroup's XCD slot (blockIdx mod kQueues) first,
// then the others in turn; it exits once every queue's cursor has passed the
// queue's length, so every wavefront terminates.
template <int U, bool CULL, bool COUNT, int KSET>
__global__ __launch_bounds__(kBlock) void k_nav_persistent(const VolumeRec *__restrict__ vols,
                                                           const DaughterRec *__restrict__ dau_all,
                                                           const CullRec *__restrict__ cul_all,
                                                           const Tile *__restrict__ tiles,
                                                           int32_t ntiles, unsigned int *cursors,
                                                           TracksDev t, double *__restrict__ step,
                                                           int32_t *__restrict__ hit,
                                                           unsigned long long *census) {
    const int lane = threadIdx.x & 63;
    __shared__ NavScratch<U> scr[CULL ? kBlock / 64 : 1];
    NavScratch<U> *my = &scr[CULL ? (threadIdx.x >> 6) : 0];
    const int home = (int)(blockIdx.x % kQueues);
    for (int qq = 0; qq < kQueues; ++qq) {
        const int q = (home + qq) % kQueues;
        const unsigned int count = ntiles > q ? (unsigned int)((ntiles - q + kQueues - 1) / kQueues) : 0u;
        for (;;) {
            unsigned int id = 0;
            if (lane == 0) id = atomicAdd(&cursors[q * kQueueStride], 1u);
            id = (unsigned int)__builtin_amdgcn_readfirstlane((int)id);
            if (id >= count) break;
            run_tile<U, CULL, COUNT, KSET>(tiles[q + kQueues * (int64_t)id], vols, dau_all, cul_all, t,
                                           step, hit, census, lane, my);
        }
    }
}

// Hardware-scheduled form: one wavefront per tile, workgroups dispatched in
// tile order (same parameters as the persistent form; `cursors` unused).
// Every kind: held to 5 wavefronts per SIMD as the basket navigator (up to
// 4 rounds per wavefront; with 8 the LDS allows 3 anyway).
template <int U, bool CULL, bool COUNT, int KSET>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(KSET == kSetAll && U <= 4 ? 5 : 1))) void k_nav_tiles(const VolumeRec *__restrict__ vols,
                                                      const DaughterRec *__restrict__ dau_all,
                                                      const CullRec *__restrict__ cul_all,
                                                      const Tile *__restrict__ tiles, int32_t ntiles,
                                                      unsigned int *cursors, TracksDev t,
                                                      double *__restrict__ step,
                                                      int32_t *__restrict__ hit,
                                                      unsigned long long *census) {
    (void)cursors;
    __shared__ NavScratch<U> scr[CULL ? kBlock / 64 : 1];
    const int w = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6)));
    if constexpr (CULL && !COUNT && KSET != kSetBasic) {
        // volumes of more kinds: the workgroup's wavefronts pool their last
        // flush when their four tiles belong to one volume (work of about
        // the same length: tiles of one volume come together in the cost
        // order); a wavefront past the last tile takes part with no tracks
        __shared__ PoolInfo<kBlock / 64> pool;
        const int w0 = (int)blockIdx.x * (kBlock / 64);
        bool shared = w0 + kBlock / 64 <= ntiles;
        for (int q = 1; shared && q < kBlock / 64; ++q) shared = tiles[w0 + q].volume == tiles[w0].volume;
        Tile tl;
        tl.volume = 0;
        tl.count = 0;
        tl.offset = 0;
        if (w < ntiles) tl = tiles[w];
        const VolumeRec &v = vols[tl.volume];
        nav_compact_pooled<U, kBlock / 64, false, false, KSET>(v, dau_all, cul_all, v.first, nullptr, t, tl.offset,
                                                               tl.count, scr, pool, shared, (int)(threadIdx.x >> 6),
                                                               (int)(threadIdx.x & 63), step, hit, nullptr);
        return;
    }
    if (w >= ntiles) return;
    run_tile<U, CULL, COUNT, KSET>(tiles[w], vols, dau_all, cul_all, t, step, hit, census,
                                   (int)(threadIdx.x & 63), &scr[CULL ? (threadIdx.x >> 6) : 0]);
}

// Expands the (cost-sorted) basket list into tiles of at most tile_n tracks:
// basket b owns tiles [tile_start[b], tile_start[b + 1]). The baskets are
// split into one contiguous run per wavefront (ceil(nb / waves) baskets, so
// a few hundred baskets spread over as many wavefronts); within its run a
// wavefront reads up to 64 basket records at once, lane j taking record j
// (mapped host memory: one round trip per 64), then writes each basket's
// tiles 64 at a time. Also resets the persistent kernel's queue cursors.
__global__ __launch_bounds__(kBlock) void k_build_tiles(BuildTilesArgs a) {
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const int nwaves = gridDim.x * (kBlock / 64);
    if (blockIdx.x == 0 && threadIdx.x < kQueues) a.cursors[threadIdx.x * kQueueStride] = 0u;
    const int run = (a.nb + nwaves - 1) / nwaves;
    const int b0 = wave * run;
    const int b1 = b0 + run < a.nb ? b0 + run : a.nb;
    for (int base = b0; base < b1; base += 64) {
        const int b = base + lane;
        int vol = 0;
        int64_t off = 0, n = 0, first = 0, last = 0;
        if (b < b1) {
            const BasketRec bk = a.baskets[b];
            vol = bk.volume;
            off = bk.offset;
            n = bk.n;
            first = a.tile_start[b];
            last = a.tile_start[b + 1];
        }
        const int m = b1 - base < 64 ? b1 - base : 64;
        for (int i = 0; i < m; ++i) {
            const int v_i = __shfl(vol, i);
            const int64_t off_i = __shfl(off, i), n_i = __shfl(n, i);
            const int64_t f_i = __shfl(first, i), l_i = __shfl(last, i);
            for (int64_t c = lane; c < l_i - f_i; c += 64) {
                const int64_t o = c * a.tile_n;
                const int64_t left = n_i - o;
                Tile tl;
                tl.volume = v_i;
                tl.count = (int32_t)(left < a.tile_n ? left : a.tile_n);
                tl.offset = off_i + o;
                a.tiles[f_i + c] = tl;
            }
        }
    }
}

template <int U, bool CULL, bool COUNT, int KSET>
static const void *pick_mode(bool persistent) {
    return persistent ? reinterpret_cast<const void *>(&k_nav_persistent<U, CULL, COUNT, KSET>)
                      : reinterpret_cast<const void *>(&k_nav_tiles<U, CULL, COUNT, KSET>);
}

template <bool CULL, bool COUNT, int KSET>
static const void *pick_u(int U, bool persistent) {
    switch (U) {
        case 1: return pick_mode<1, CULL, COUNT, KSET>(persistent);
        case 2: return pick_mode<2, CULL, COUNT, KSET>(persistent);
        case 4: return pick_mode<4, CULL, COUNT, KSET>(persistent);
        default: return pick_mode<8, CULL, COUNT, KSET>(persistent);
    }
}

// The census variants (instrumentation, not timed) exist for the full kind
// set only.
const void *batched_kernel(int tracks_per_lane, bool cull, bool persistent, bool count, int kset) {
    const void *k = nullptr;
    if (count) {
        k = cull ? pick_u<true, true, kSetAll>(tracks_per_lane, persistent)
                 : pick_u<false, true, kSetAll>(tracks_per_lane, persistent);
    } else if (cull) {
        GN_KSET(kset, (k = pick_u<true, false, KS>(tracks_per_lane, persistent)));
    } else {
        GN_KSET(kset, (k = pick_u<false, false, KS>(tracks_per_lane, persistent)));
    }
    return k;
}

const void *build_tiles_kernel() { return reinterpret_cast<const void *>(&k_build_tiles); }

int batched_grid(int waves_per_simd, int num_cus, int64_t ntiles) {
    // persistent: 4 SIMDs per CU and kBlock / 64 = 4 wavefronts per workgroup,
    // so num_cus * waves_per_simd workgroups give waves_per_simd per SIMD;
    // hardware-scheduled: one wavefront per tile
    if (waves_per_simd > 0) return num_cus * waves_per_simd;
    return (int)((ntiles + kBlock / 64 - 1) / (kBlock / 64));
}

// ------------------------------------------------------------------ adjoint
// The volume's culling records moved by this call's daughter offsets, for
// the adjoint's forward: centre T' = T + offset and the threshold of the
// expanded test for it, q' = r2 - |T'|^2 + 64 eps (3 R + 2 |T'|)^2 (R the
// mother's bounding radius), the same bound as the unshifted records'.
// Padding records are copied (q = -infinity: they never pass). The moved
// centre differs from T + offset by a rounding, far inside the culling
// radius's enlargement of 1e-6 relative + 1e-6, so the tests stay
// conservative for the daughter where the queued pairs place it.
__global__ __launch_bounds__(kBlock) void k_shift_cull(const VolumeRec *__restrict__ vol,
                                                       const CullRec *__restrict__ cul,
                                                       const DaughterRec *__restrict__ dau,
                                                       const double *__restrict__ offs,
                                                       CullRec *__restrict__ out) {
    const int nd = vol->nd;
    const int ndp = (nd + kCullChunk - 1) / kCullChunk * kCullChunk;
    const double R = vol->bound_r;
    for (int k = (int)(blockIdx.x * blockDim.x + threadIdx.x); k < ndp; k += (int)(gridDim.x * blockDim.x)) {
        if (k < nd) {
            const double tx = cul[k].tx + offs[3 * k + 0];
            const double ty = cul[k].ty + offs[3 * k + 1];
            const double tz = cul[k].tz + offs[3 * k + 2];
            const double tt = tx * tx + ty * ty + tz * tz;
            const double span = 3.0 * R + 2.0 * fsqrt(tt);
            out[k] = CullRec{tx, ty, tz, dau[k].cull_r2 - tt + 64.0 * 2.220446049250313e-16 * span * span};
        } else {
            out[k] = cul[k];
        }
    }
}

// For each track: recompute the forward step keeping the surface that set it,
// take that surface's normal n (mother frame) at the hit point and, by the
// implicit-function theorem on the surface equation,
//   ds/dp = -n / (n.d),  ds/dd = s ds/dp,  ds/d delta_hit = n / (n.d).
// With phi = gstep s + ghit . (p + s d) and c = gstep + ghit . d:
//   g_p = ghit + c ds/dp,  g_d = s ghit + c ds/dd,  g_delta_hit += c ds/d delta.
// The offset gradient of the workgroup's tracks is summed per daughter in a
// fixed lane order into the workgroup's row of `partial`, accumulated over
// the workgroup's passes in LDS when lds_acc (3 nd doubles; else in the row
// itself) and written once. With SHIFTED the forward's culling tests read
// `shifted` (k_shift_cull), the records moved by the offsets.
template <bool HAS_OFFS, bool CULL, int KSET, bool SHIFTED = false>
__global__ __launch_bounds__(kBlock) void k_nav_backward(
    const VolumeRec *__restrict__ vol, const DaughterRec *__restrict__ dau,
    const CullRec *__restrict__ cul, TracksDev t, const double *__restrict__ offs,
    const double *__restrict__ gstep,
    const double *__restrict__ ghit, double *__restrict__ g_o, double *__restrict__ g_d,
    double *__restrict__ partial, bool lds_acc, const CullRec *__restrict__ shifted) {
    __shared__ double s_g[3][kBlock];
    __shared__ NavScratch<1> scr[CULL ? kBlock / 64 : 1];
    // [3 nd] doubles of the row's accumulator when lds_acc, then 4 nd + nd + 1
    // ints (see below)
    extern __shared__ double s_dyn[];
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int nd = vol->nd;
    const int nj = 3 * nd;
    double *prow = partial ? partial + (size_t)blockIdx.x * nj : nullptr;
    double *acc_row = lds_acc ? s_dyn : prow;  // each entry j is thread (j mod kBlock)'s alone
    int *s_bins = reinterpret_cast<int *>(s_dyn + (lds_acc ? nj : 0));
    if (prow)
        for (int j = tid; j < nj; j += kBlock) acc_row[j] = 0.0;
    const int64_t n = t.n;
    for (int64_t base = (int64_t)blockIdx.x * kBlock; base < n; base += (int64_t)gridDim.x * kBlock) {
        const int64_t i = base + tid;
        int h = -2;
        double gdx = 0.0, gdy = 0.0, gdz = 0.0;
        if constexpr (CULL) {
            // the forward step and hit by the compacted navigator (per
            // wavefront of 64 tracks)
            const int64_t wbase = base + wave * 64;
            if (wbase < n) {
                const int cnt = n - wbase < 64 ? (int)(n - wbase) : 64;
                if (SHIFTED)
                    nav_compact_core<1, HAS_OFFS, false, KSET, true, true, SHIFTED>(
                        *vol, dau, cul, offs, t, wbase, cnt, scr[wave], lane, nullptr, shifted);
                else
                    nav_compact_core<1, HAS_OFFS, false, KSET>(*vol, dau, cul, offs, t, wbase, cnt, scr[wave],
                                                               lane);
            }
        }
        if (i < n) {
            const double x = t.x[i], y = t.y[i], z = t.z[i];
            const double ux = t.ux[i], uy = t.uy[i], uz = t.uz[i];
            double best;
            int sid;
            if constexpr (CULL) {
                // the step, the winner and the surface that set its step, as
                // the compacted navigator left them
                best = key_step(lds_load(&scr[wave].key[lane]));
                const int v = lds_load(&scr[wave].hit[lane]);
                h = hit_index(v);
                sid = hit_surface(v);
            } else {
                nav_track<HAS_OFFS, true, false, KSET>(*vol, dau, cul, offs, x, y, z, ux, uy, uz, best,
                                                       h, sid);
            }
            const bool finite = best < kBig;
            const double s = finite ? best : 0.0;
            const double hx = fma(s, ux, x), hy = fma(s, uy, y), hz = fma(s, uz, z);
            double nx, ny, nz;
            if (h < 0) {
                surface_normal(vol->mother, vol->pcon, sid, hx, hy, hz, nx, ny, nz);
            } else {
                const DaughterRec &D = dau[h];
                double wx = hx - D.tr[0], wy = hy - D.tr[1], wz = hz - D.tr[2];
                if (HAS_OFFS) {
                    wx -= offs[3 * h + 0];
                    wy -= offs[3 * h + 1];
                    wz -= offs[3 * h + 2];
                }
                const double *R = D.rot;
                const double lx = fma(R[6], wz, fma(R[3], wy, R[0] * wx));
                const double ly = fma(R[7], wz, fma(R[4], wy, R[1] * wx));
                const double lz = fma(R[8], wz, fma(R[5], wy, R[2] * wx));
                double mx, my, mz;
                surface_normal(D.shape, D.pcon, sid, lx, ly, lz, mx, my, mz);
                // back to the mother frame: n = R m
                nx = fma(R[2], mz, fma(R[1], my, R[0] * mx));
                ny = fma(R[5], mz, fma(R[4], my, R[3] * mx));
                nz = fma(R[8], mz, fma(R[7], my, R[6] * mx));
            }
            const double nd_ = fma(nz, uz, fma(ny, uy, nx * ux));
            const bool ok = finite && best > 0.0 && nd_ != 0.0;
            const double inv = ok ? -1.0 / nd_ : 0.0;
            const double dsx = nx * inv, dsy = ny * inv, dsz = nz * inv;  // ds/dp
            const double gs = gstep ? gstep[i] : 0.0;
            double ghx = 0.0, ghy = 0.0, ghz = 0.0;
            if (ghit) {
                ghx = ghit[i];
                ghy = ghit[n + i];
                ghz = ghit[2 * n + i];
            }
            const double c = fma(ghz, uz, fma(ghy, uy, fma(ghx, ux, gs)));
            if (g_o) {
                g_o[i] = fma(c, dsx, ghx);
                g_o[n + i] = fma(c, dsy, ghy);
                g_o[2 * n + i] = fma(c, dsz, ghz);
            }
            if (g_d) {
                const double cs = c * s;
                g_d[i] = fma(cs, dsx, s * ghx);
                g_d[n + i] = fma(cs, dsy, s * ghy);
                g_d[2 * n + i] = fma(cs, dsz, s * ghz);
            }
            gdx = -c * dsx;
            gdy = -c * dsy;
            gdz = -c * dsz;
        }
        if (prow) {
            // Offset gradient of the workgroup's tracks per daughter: a
            // stable counting sort of the contributions by hit daughter,
            // then each (daughter, component) sums its run in track order,
            // the order of a plain scan over the workgroup's tracks.
            int *cnt = s_bins;           // [4][nd]: per-wavefront counts
            int *run = s_bins + 4 * nd;  // [nd + 1]: start of each daughter's run
            // each wavefront clears its own row (the other wavefronts last
            // read it before the barrier that ended the previous pass), then
            // counts its tracks per daughter and ranks each among the
            // earlier lanes with the same daughter
            for (int k = lane; k < nd; k += 64) cnt[wave * nd + k] = 0;
            int rank = 0;
            unsigned long long rem = __builtin_amdgcn_ballot_w64(h >= 0);
            while (rem != 0ull) {
                const int k = __builtin_amdgcn_readlane(h, __ffsll((long long)rem) - 1);
                const unsigned long long m = __builtin_amdgcn_ballot_w64(h == k);
                if (h == k) rank = lanes_below(m);
                if (lane == 0) cnt[wave * nd + k] = __popcll(m);
                rem &= ~m;
            }
            __syncthreads();
            // every wavefront forms the runs itself (an exclusive scan of the
            // daughters' totals, 64 daughters a pass, lane = daughter) and
            // its own offset within each run; wavefront 0 publishes the runs
            int pos = 0;
            int carry = 0;
            for (int k0 = 0; k0 < nd; k0 += 64) {
                const int k = k0 + lane;
                int tot = 0, below = 0;
                if (k < nd) {
#pragma unroll
                    for (int w = 0; w < kBlock / 64; ++w) {
                        const int c = cnt[w * nd + k];
                        tot += c;
                        below += w < wave ? c : 0;
                    }
                }
                int incl = tot;
                for (int dlt = 1; dlt < 64; dlt <<= 1) {
                    const int v = __shfl_up(incl, dlt);
                    if (lane >= dlt) incl += v;
                }
                const int start = carry + incl - tot;
                if (wave == 0 && k < nd) run[k] = start;
                // a lane whose daughter falls in this pass takes its offset
                const int off = __shfl(start + below, (h - k0) & 63);
                if (h >= k0 && h < k0 + 64) pos = off + rank;
                carry += __shfl(incl, 63);
            }
            if (wave == 0 && lane == 0) run[nd] = carry;
            if (h >= 0) {
                s_g[0][pos] = gdx;
                s_g[1][pos] = gdy;
                s_g[2][pos] = gdz;
            }
            __syncthreads();
            for (int j = tid; j < nj; j += kBlock) {
                const int k = j / 3, comp = j - 3 * k;
                double acc = 0.0;
                for (int q = run[k]; q < run[k + 1]; ++q) acc += s_g[comp][q];
                acc_row[j] += acc;
            }
            __syncthreads();
        }
    }
    if (prow && lds_acc)
        for (int j = tid; j < nj; j += kBlock) prow[j] = acc_row[j];
}

// out[j] = sum over workgroups b of partial[b][j], in a fixed order.
__global__ __launch_bounds__(kBlock) void k_reduce_partials(const double *__restrict__ partial,
                                                            int nblocks, int nj,
                                                            double *__restrict__ out) {
    __shared__ double s[kBlock];
    const int j = blockIdx.x;
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += kBlock) acc += partial[(size_t)b * nj + j];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[j] = s[0];
}

constexpr int kBackwardLdsAcc = 256;

template <bool CULL, int KSET>
static void launch_backward_variant(int nblocks, int nd, const VolumeRec *vol, const DaughterRec *dau,
                                    const CullRec *cul, const TracksDev &t, const double *offs, const double *gstep,
                                    const double *ghit, double *g_o, double *g_d, double *part,
                                    const CullRec *shifted, hipStream_t st) {
    // the offset-gradient sort's counts and runs; the row's accumulator in
    // LDS up to kBackwardLdsAcc daughters (6 KB)
    const bool lds_acc = part && nd <= kBackwardLdsAcc;
    const size_t dyn = (lds_acc ? sizeof(double) * 3 * (size_t)nd : 0) + sizeof(int) * (size_t)(5 * nd + 1);
    if (offs && CULL && shifted)
        hipLaunchKernelGGL((k_nav_backward<true, CULL, KSET, CULL>), dim3(nblocks), dim3(kBlock), dyn, st, vol, dau,
                           cul, t, offs, gstep, ghit, g_o, g_d, part, lds_acc, shifted);
    else if (offs)
        hipLaunchKernelGGL((k_nav_backward<true, CULL, KSET>), dim3(nblocks), dim3(kBlock), dyn, st, vol, dau, cul, t,
                           offs, gstep, ghit, g_o, g_d, part, lds_acc, nullptr);
    else
        hipLaunchKernelGGL((k_nav_backward<false, CULL, KSET>), dim3(nblocks), dim3(kBlock), dyn, st, vol, dau, cul, t,
                           offs, gstep, ghit, g_o, g_d, part, lds_acc, nullptr);
}

int backward_blocks(int64_t n) {
    const int64_t need = (n + kBlock - 1) / kBlock;
    return (int)(need < kBackwardMaxBlocks ? (need > 0 ? need : 1) : kBackwardMaxBlocks);
}

hipError_t launch_backward(const VolumeRec *vol, const DaughterRec *dau, const CullRec *cul, int nd,
                           const TracksDev &t, const double *offs, const double *gstep,
                           const double *ghit, double *g_o, double *g_d, double *partial,
                           double *g_off, bool cull, int kset, CullRec *shift_buf, hipStream_t st) {
    const int nblocks = backward_blocks(t.n);
    double *part = (g_off && nd > 0) ? partial : nullptr;
    if (t.n > 0 || part) {
        const CullRec *shifted = nullptr;
        if (cull && offs && shift_buf && nd > 0 && t.n > 0) {
            const int ndp = (nd + kCullChunk - 1) / kCullChunk * kCullChunk;
            hipLaunchKernelGGL(k_shift_cull, dim3((ndp + kBlock - 1) / kBlock), dim3(kBlock), 0, st, vol, cul, dau,
                               offs, shift_buf);
            shifted = shift_buf;
        }
        if (cull)
            GN_KSET(kset, (launch_backward_variant<true, KS>(nblocks, nd, vol, dau, cul, t, offs, gstep, ghit,
                                                             g_o, g_d, part, shifted, st)));
        else
            GN_KSET(kset, (launch_backward_variant<false, KS>(nblocks, nd, vol, dau, cul, t, offs, gstep, ghit,
                                                              g_o, g_d, part, nullptr, st)));
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (part) {
        hipLaunchKernelGGL(k_reduce_partials, dim3(3 * nd), dim3(kBlock), 0, st, part, nblocks, 3 * nd,
                           g_off);
        return hipGetLastError();
    }
    return hipSuccess;
}

// ------------------------------------------------ allocation-free adjoint
// The offset gradient's per-workgroup partial sums for the adjoint entry
// point that allocates nothing: a file-scope device array, one copy per GPU
// the library runs on, held until the process ends. In host code the name
// `scratch` is a host-side stand-in, not a device address: host code uses
// only the address hipGetSymbolAddress returns for the current device,
// looked up at the first call on each device and kept.
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t scratch_partials(double **out) {
    *out = nullptr;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace gn

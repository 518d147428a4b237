// Host-side interface between the C ABI (geonav_abi.cpp) and the kernel
// launchers (geonav_kernels.hip). Not part of the public header.
#pragma once

#include <hip/hip_runtime.h>

#include "geonav_device.hpp"

namespace gn {

constexpr int kBlock = 256;          // threads per workgroup (4 wavefronts)
constexpr int kBackwardMaxBlocks = 2048;

hipError_t launch_shape_query(const ShapeRec &s, const PconRec &pc, int query, const TracksDev &t,
                              void *out, hipStream_t st);

hipError_t launch_nav_basket(const VolumeRec *vol, const DaughterRec *dau, const CullRec *cul,
                             const TracksDev &t, const double *offs, double *step, int32_t *hit,
                             double *hitpt, bool cull, int kset, hipStream_t st);

hipError_t launch_nav_safety(const VolumeRec *vol, const DaughterRec *dau, const CullRec *cul,
                             const TracksDev &t, const double *offs, double *out, bool cull,
                             int kset, hipStream_t st);
hipError_t launch_nav_locate(const VolumeRec *vol, const DaughterRec *dau, const CullRec *cul,
                             const TracksDev &t, const double *offs, int32_t *out, bool cull,
                             int kset, hipStream_t st);

// Tile queues of the persistent batched kernel: one per XCD, cursors 256 B
// apart.
constexpr int kQueues = 8;
constexpr int kQueueStride = 64;  // in unsigned ints

// Arguments of the batched kernels, in kernel-parameter order (graph kernel
// nodes pass a pointer to each). The queue cursors are reset by
// k_build_tiles, which runs just before in the same graph.
struct PersistentArgs {
    const VolumeRec *vols;
    const DaughterRec *dau;
    const CullRec *cul;
    const Tile *tiles;
    int32_t ntiles;
    unsigned int *cursors;       // kQueues * kQueueStride
    TracksDev t;
    double *step;
    int32_t *hit;
    unsigned long long *census;  // NULL except in the census launch
};

// A basket as the device sees it (sorted by decreasing per-track cost).
struct BasketRec {
    int32_t volume;
    int32_t pad;
    int64_t offset;
    int64_t n;
};

struct BuildTilesArgs {
    const BasketRec *baskets;
    const int64_t *tile_start;  // nb + 1 prefix offsets into tiles
    int32_t nb;
    int32_t tile_n;             // tracks per tile (64 * tracks per lane)
    Tile *tiles;
    unsigned int *cursors;
};

constexpr int kBuildTilesBlocks = 256;

// Kernel function handles (for graph kernel nodes and hipLaunchKernel).
// persistent: k_nav_persistent, else k_nav_tiles (one wavefront per tile);
// count: the variant that fills the work census; kset: the kinds the
// geometry holds (kSetBasic, kSetSeg or kSetAll).
const void *batched_kernel(int tracks_per_lane, bool cull, bool persistent, bool count, int kset);
const void *build_tiles_kernel();
// Workgroups of a batched launch: num_cus * waves_per_simd (persistent) or
// one wavefront per tile (waves_per_simd == 0).
int batched_grid(int waves_per_simd, int num_cus, int64_t ntiles);

// Workgroups of an adjoint launch over n tracks (each writes one row of
// 3 * nd partial sums of the offset gradient).
int backward_blocks(int64_t n);

// The static partial-sum buffer of the allocation-free adjoint: doubles it
// holds, and its device address on the current device (looked up once per
// device).
constexpr size_t kScratchDoubles = (size_t)kBackwardMaxBlocks * 3 * 64;  // 3 MiB
hipError_t scratch_partials(double **out);

// shift_buf: room for the volume's culling records (nd rounded up to whole
// chunks) moved by the offsets, written by a small kernel before the adjoint
// when culling with offsets; NULL to cull with the offsets applied in every
// test instead.
hipError_t launch_backward(const VolumeRec *vol, const DaughterRec *dau, const CullRec *cul, int nd,
                           const TracksDev &t, const double *offs, const double *gstep,
                           const double *ghit, double *g_o, double *g_d, double *partial,
                           double *g_off, bool cull, int kset, CullRec *shift_buf, hipStream_t st);

}  // namespace gn

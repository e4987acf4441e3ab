// Internal declarations shared by the kernels (rsf_kernels.hpp / .hip) and
// the C-ABI host code (rsf_api.hip).  gfx950 only.
//
// Every pass runs over a batch of tiles (independent volumes); a single
// volume is a batch of one.  A pass launches one grid for the whole batch:
// each tile owns a contiguous range of the pass's workgroups, found from a
// prefix table, so uneven tiles share one launch.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <type_traits>

namespace rsf {

constexpr int kMaxR = 16;          // largest Gaussian radius (sigma <= 16/3)
constexpr int kXcds = 8;           // accelerator complex dies, each with its own L2
constexpr int kThreads = 256;      // z pass block: consecutive columns
constexpr int kUx = 64;            // update pass: columns per block along x
constexpr int kUy = 8;             // update pass: columns per block along y
constexpr int kUThreads = kUx * kUy;
// Largest xy plane (voxels): every in-slice byte offset of an 8-byte
// element, with a workgroup's overhang, fits a 32-bit unsigned offset.
constexpr int64_t kMaxPlane = (int64_t)1 << 28;

// Image/storage combinations other than (F32, F32) are built for radii
// kMinRMixed..kMaxRMixed.
constexpr int kMinRMixed = 4;
constexpr int kMaxRMixed = 12;

// Sampled, truncated, unit-sum Gaussian taps w[k + R], k = -R..R.
struct Taps {
    float w[2 * kMaxR + 1];
};

struct Grid3 {
    int nx, ny, nz;
    int64_t sxy;  // nx * ny
};

// How each pass cuts a tile into workgroups: row chunks of the xy passes,
// z chunks of the stage-1 z pass and of the update pass.
struct Split {
    int xy, z, u;
};

// One tile of a batch as the kernels see it (device pointers).
struct TileDesc {
    Grid3 g;
    Split sp;
    const void *I;          // image, in the image type
    float *phi[2];          // phi ping-pong: [0] the caller's buffer, [1] workspace
    void *P, *Q;            // interleaved pair fields, storage type
    void *KI;               // K * I, storage type
    void *K2I, *K2I2;       // K2 * I and K2 * I^2 (Sec. 4.2 force, sigma2 > 0), storage type
    float *cx, *cy, *cz;    // K * 1 = cx[x] cy[y] cz[z]
    double *partials;       // one sum |dphi| per update-pass block
    double *hist;           // sum |dphi| per iteration run
    int hist_cap;           // entries of hist = iterations asked of this tile
    int *flags;             // [0] 0 running, 1 stopped by tol, 2 done; [1] iterations run
    // one-step probe outputs (float fields), null when unused
    float *probe_H, *probe_f1, *probe_f2, *probe_Fd, *probe_kappa, *probe_lap, *probe_R,
        *probe_E;
};

// Scalars shared by every tile of a batch.
struct Coeffs {
    float l1, l2, nu, mu, dt;
    float eps, eps_over_pi, eps2;   // delta = eps_over_pi / (eps2 + phi^2)
    float eta;
    int reg;                        // 0 double well, 1 single well
    int force;                      // 0 RSF e_i (sigma), 1 Sec. 4.2 form (sigma2)
    int square;                     // XY_ONE: convolve I^2 instead of I
    double tol;                     // stop a tile once sum|dphi| / voxels < tol (0: never)
};

// A pass over a batch: the tiles and the pass's workgroup prefix table (n + 1
// entries: tile t owns workgroups [start[t], start[t+1])).  A tile's current
// iterate n (flags[1]) is in phi[n & 1], so tiles of one batch may be at
// different iterations.
//
// Workgroups are dispatched to the XCDs round robin (hardware workgroup b on
// XCD b % 8).  XCD k takes the contiguous range [xcd[k], xcd[k+1]) of the
// batch's workgroups, the ranges cut for equal estimated cost; the grid is 8
// times the longest range and the surplus workgroups exit at once.
struct Batch {
    const TileDesc *tiles;
    const int *start;
    int n;
    int xcd[kXcds + 1];
};

// Workgroup counts of one tile under a split.
__host__ __device__ inline int nbx64(int nx) { return (nx + 63) / 64; }
__host__ __device__ inline int64_t xy_blocks(const Grid3 &g, const Split &s)
{
    return (int64_t)nbx64(g.nx) * s.xy * g.nz;
}
// z passes: workgroups of kThreads consecutive columns (y nx + x) times a z
// chunk.
__host__ __device__ inline int64_t z_cols(const Grid3 &g) { return (g.sxy + kThreads - 1) / kThreads; }
__host__ __device__ inline int64_t z_blocks(const Grid3 &g, const Split &s)
{
    return z_cols(g) * s.z;
}
__host__ __device__ inline int64_t u_blocks(const Grid3 &g, const Split &s)
{
    return (int64_t)((g.nx + kUx - 1) / kUx) * ((g.ny + kUy - 1) / kUy) * s.u;
}

// Workgroups a whole batch aims at per pass: xy waves, z-pass workgroups,
// update-pass workgroups.
struct Targets {
    int64_t xy, z, u;
};
constexpr Targets kDefaultTargets{16384, 2048, 1024};

// Split of one volume aiming at the given workgroup counts per pass (the
// autotuner varies them); every chunk is non-empty and at least 8 long.
Split make_split(const Grid3 &g, int64_t xy_waves, int64_t z_target, int64_t u_target);
// Split of a tile holding fraction `share` of its batch's voxels: that share
// of the batch's targets.
Split default_split(const Grid3 &g, double share = 1.0, const Targets &tg = kDefaultTargets);
// Split of a single volume from the resident capacity of the z and update
// passes (R: Gaussian radius): z chunks are chosen so that the launches' last
// round of workgroups is not left nearly empty.
Split capacity_split(const Grid3 &g, int R);
// Workgroups the GPU keeps resident at once: z passes (256-thread groups at
// 8 per CU) and the update pass (512-thread groups at 2 per CU), on 256 CUs.
constexpr int64_t kResidentZ = 2048;
constexpr int64_t kResidentU = 512;
// Update-pass workgroups of a tile under any valid split are at most this.
__host__ __device__ inline int64_t u_blocks_max(const Grid3 &g)
{
    return (int64_t)((g.nx + kUx - 1) / kUx) * ((g.ny + kUy - 1) / kUy) * ((g.nz + 7) / 8);
}
bool split_valid(const Grid3 &g, const Split &s);

bool types_supported(int R, int image_dtype, int storage_dtype);

// xy pass modes: XY_ONE reads the image (or its square) and writes one field
// (P), for K*I; XY_FITS reads the pair P and K*I and writes the pair Q;
// XY_TWO reads the pair Q and writes the pair P; XY_PAPER reads the pair P,
// K*I and the image and writes the Sec. 4.2 force with sigma2 = 0 to Q as
// float; XY_PAPER2 reads K2*I and K2*I^2 in place of the image (sigma2 > 0).
enum XyMode { XY_ONE = 0, XY_TWO = 1, XY_FITS = 2, XY_PAPER = 3, XY_PAPER2 = 4 };
// Where the plain z pass writes: K*I, K2*I or K2*I^2.
enum ZTarget { Z_TO_KI = 0, Z_TO_K2I = 1, Z_TO_K2I2 = 2 };

// One workgroup per tile: K*1 edge tables, flags cleared.
hipError_t launch_setup(const Batch &b, const Taps &t, int R, hipStream_t s);
// A small host-built table written to device memory by a kernel from its own
// argument: no pinned staging buffer and no copy, for the entry point that
// allocates nothing.
constexpr int kTableBlobBytes = 2048;
struct TableBlob {
    uint32_t w[kTableBlobBytes / 4];
};
hipError_t launch_put_table(void *dst, const TableBlob &blob, int bytes, hipStream_t s);
hipError_t launch_xy(int R, int mode, int image_dtype, int storage_dtype, const Batch &b,
                     int64_t blocks, const Taps &t, const Coeffs &c, bool probe, hipStream_t s);
// K*I: the z pass of P into KI.
hipError_t launch_z_plain(int R, int storage_dtype, const Batch &b, int64_t blocks,
                          const Taps &t, int target, hipStream_t s);
// Stage-1 z pass: (phi, I) -> the pair P = (Kz*(H I), Kz*H).
hipError_t launch_z_heaviside(int R, int image_dtype, int storage_dtype, const Batch &b,
                              int64_t blocks, const Taps &t, const Coeffs &c, bool probe,
                              hipStream_t s);
// Stage-2 z pass of the pair P = (Kxy*g1, Kxy*g2) and the update into the
// other phi buffer, with per-block |dphi| partial sums.
hipError_t launch_z_update(int R, int image_dtype, int storage_dtype, const Batch &b,
                           int64_t blocks, const Taps &t, const Coeffs &c, bool probe,
                           hipStream_t s);
// The update reading the Sec. 4.2 force (sigma2 = 0) that XY_PAPER wrote.
hipError_t launch_z_update_paper(int image_dtype, int storage_dtype, const Batch &b,
                                 int64_t blocks, const Coeffs &c, bool probe, hipStream_t s);
// Largest Gaussian radius whose RSF-force update is fused with the next
// stage-1 pass (the Sec. 4.2 force's update has no stage-2 ring: any radius).
// A stage-2 ring slot holds two floats with FP32 or BF16 storage and one
// packed pair with FP16 storage, which leaves room for the stage-1 ring and
// the prefetched stage with no spill in the march up to radius 9 (8 with a
// uint16 image), resp. 12 (storage and image dtypes as in rsf_dtype: 1 is
// FP16, 3 uint16).
constexpr int kFuseMaxR = 9;
constexpr int kFuseMaxRU16 = 8;
constexpr int kFuseMaxRPacked = 12;
template <class ST, class IT>
constexpr int fuse_max_r_t = std::is_same<ST, _Float16>::value
                                 ? kFuseMaxRPacked
                                 : (std::is_same<IT, uint16_t>::value ? kFuseMaxRU16 : kFuseMaxR);
inline int fuse_max_r(int storage_dtype, int image_dtype)
{
    return storage_dtype == 1 ? kFuseMaxRPacked : (image_dtype == 3 ? kFuseMaxRU16 : kFuseMaxR);
}
// The update (RSF force, or the Sec. 4.2 force if `paper`) fused with the
// next iteration's stage-1 z pass (writes P from phi' as launch_z_heaviside
// would); every tile marched whole in z.
hipError_t launch_z_update_fused(int R, int image_dtype, int storage_dtype, const Batch &b,
                                 int64_t blocks, const Taps &t, const Coeffs &c, bool paper,
                                 hipStream_t s);
// One workgroup per tile: fixed-order FP64 sum of the partials; counts the
// iteration and stops the tile at its tolerance or its last iteration.
hipError_t launch_reduce(const Batch &b, const Coeffs &c, hipStream_t s);
// Copy an odd final iterate from phi[1] to phi[0] (workgroups of the z pass).
hipError_t launch_finish(const Batch &b, int64_t blocks, hipStream_t s);

// Volume-level driver (Sec. 4.1): one sub-volume box of a large volume.
struct SubBox {
    int lo[3], ext[3];              // x, y, z origin and extent in the volume
    int core_lo[3], core_hi[3];     // its core (the part it owns outright)
    int nb_lo[3], nb_hi[3];         // 1 when a neighbour shares the face
};
// Copy box `b` of the volume (elements of elem_bytes, 2 or 4) into a dense
// tile buffer.
hipError_t launch_gather(const void *src, void *dst, int elem_bytes, int64_t nx, int64_t ny,
                         const SubBox &b, hipStream_t s);
// acc += w * tile over box b, w the product of per-axis linear ramps across
// the 2C-wide overlaps with the box's neighbours (the curtain).
hipError_t launch_merge(float *acc, const float *tile, int64_t nx, int64_t ny, const SubBox &b,
                        int curtain, hipStream_t s);
hipError_t launch_fill(float *dst, int64_t n, float v, hipStream_t s);

// Initialisation (Sec. 4.3).  Slices smoothed by the 2D Gaussian (x pass from
// the image, then y pass), the determinant and trace of the in-slice Hessian
// with per-workgroup maxima of the determinant, the seed mask, and one fast
// sweeping hyperplane.
constexpr float kFar = 1e30f;        // distance of a voxel no seed has reached
hipError_t launch_smooth_x(const void *img, int image_dtype, float *out, int64_t nx, int64_t ny,
                           int64_t nz, const Taps &t, int R, hipStream_t s);
hipError_t launch_smooth_y(const float *in, float *out, int64_t nx, int64_t ny, int64_t nz,
                           const Taps &t, int R, hipStream_t s);
// doh, trace from L; partial maxima of doh into part[blocks]; returns blocks
hipError_t launch_hessian(const float *L, float *doh, float *tr, float *part, int64_t nx,
                          int64_t ny, int64_t nz, int *blocks, hipStream_t s);
// max of part[0..n) into out[0] (one workgroup, fixed order)
hipError_t launch_max(const float *part, int n, float *out, hipStream_t s);
// mask and u (0 at seeds, kFar elsewhere); per-workgroup seed counts into cnt
hipError_t launch_seeds(const float *doh, const float *tr, const float *maxv, float threshold,
                        unsigned char *mask, float *u, unsigned *cnt, int64_t nx, int64_t ny,
                        int64_t nz, hipStream_t s);
// Fast sweeping by hyperplanes of blocks: a sweep with axis orders dir (bit
// 0: x descending, bit 1: y, bit 2: z) is sweep_block_planes() launches of
// launch_sweep_blocks with H = 0, 1, ...
int64_t sweep_block_planes(int64_t nx, int64_t ny, int64_t nz);
hipError_t launch_sweep_blocks(float *u, int64_t nx, int64_t ny, int64_t nz, int dir, int64_t H,
                               hipStream_t s);
// phi = offset - u
hipError_t launch_offset(const float *u, float *phi, int64_t n, float offset, hipStream_t s);

// Per-radius, per-type launchers behind the dispatchers (rsf_kernels.hpp).
template <int R, class IT, class ST>
hipError_t launch_xy_r(int mode, const Batch &b, int64_t blocks, const Taps &t, const Coeffs &c,
                       bool probe, hipStream_t s);
template <int R, class ST>
hipError_t launch_z_plain_r(const Batch &b, int64_t blocks, const Taps &t, int target,
                            hipStream_t s);
template <int R, class IT, class ST>
hipError_t launch_z_heaviside_r(const Batch &b, int64_t blocks, const Taps &t, const Coeffs &c,
                                bool probe, hipStream_t s);
template <int R, class IT, class ST>
hipError_t launch_z_update_r(const Batch &b, int64_t blocks, const Taps &t, const Coeffs &c,
                             bool probe, hipStream_t s);
template <class IT, class ST>
hipError_t launch_z_update_paper_r(const Batch &b, int64_t blocks, const Coeffs &c, bool probe,
                                   hipStream_t s);
template <int R, class IT, class ST>
hipError_t launch_z_update_fused_r(const Batch &b, int64_t blocks, const Taps &t, const Coeffs &c,
                                   bool paper, hipStream_t s);

}  // namespace rsf

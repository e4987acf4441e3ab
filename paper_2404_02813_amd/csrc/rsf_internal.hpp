// Internal declarations shared by the kernels (rsf_kernels.hip) and the
// C-ABI host code (rsf_api.hip).  gfx950 only.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace rsf {

constexpr int kMaxR = 16;          // largest Gaussian radius (sigma <= 16/3)
constexpr int kZx = 64;            // z pass: columns per block along x
constexpr int kZy = 4;             // z pass: columns per block along y
constexpr int kThreads = 256;      // z pass block
constexpr int kUx = 64;            // update pass: columns per block along x
constexpr int kUy = 8;             // update pass: columns per block along y
constexpr int kUThreads = kUx * kUy;

// Sampled, truncated, unit-sum Gaussian taps w[k + R], k = -R..R.
struct Taps {
    float w[2 * kMaxR + 1];
};

struct Grid3 {
    int nx, ny, nz;
    int64_t sxy;  // nx * ny
};

// Epilogue of the stage-1 xy pass: region fits and the two force-convolution
// inputs g1 = l1 f1 - l2 f2, g2 = l1 f1^2 - l2 f2^2.
struct FitArgs {
    const void *KI;               // K * I, in the storage type
    const float *cx, *cy, *cz;    // K * 1 = cx[x] cy[y] cz[z]
    float l1, l2;
    float *probe_f1, *probe_f2;   // optional
};

// Epilogue of the stage-2 z pass: force, curvature, regulariser, update.
struct UpdArgs {
    const void *I;                // image, in the image type
    const float *phi;             // phi_n
    float *phi_out;               // phi_{n+1}
    const float *cx, *cy, *cz;
    float l1, l2, nu, mu, dt;
    float eps_over_pi, eps2;      // delta = eps_over_pi / (eps2 + phi^2)
    float eta;
    int reg;                      // 0 double well, 1 single well
    double *partials;             // one sum|dphi| per block
    float *probe_Fd, *probe_kappa, *probe_lap, *probe_R, *probe_E;
};

// Number of z chunks a z pass splits the volume into (also sizes the
// per-block partial sums of the update pass).
int z_chunks(const Grid3 &g);
int64_t z_blocks(const Grid3 &g);
int u_chunks(const Grid3 &g);
int64_t u_blocks(const Grid3 &g);   // blocks (and partial sums) of the update pass
int xy_chunks(const Grid3 &g);
int xy_blocks(const Grid3 &g);

hipError_t launch_edges(float *cx, float *cy, float *cz, Grid3 g, const Taps &t, int R,
                        hipStream_t s);
hipError_t launch_flags_init(int *flags, hipStream_t s);

// Element types (values of rsf_dtype): image RSF_F32 or RSF_U16, storage of
// the intermediate fields RSF_F32, RSF_F16 or RSF_BF16.  Combinations other
// than (F32, F32) are built for radii kMinRMixed..kMaxRMixed.
constexpr int kMinRMixed = 4;
constexpr int kMaxRMixed = 12;
bool types_supported(int R, int image_dtype, int storage_dtype);

// xy pass modes: one field; two fields; two fields + region-fit epilogue.
enum XyMode { XY_ONE = 0, XY_TWO = 1, XY_FITS = 2 };
// XY_ONE reads one field of the image type and writes one field of the
// storage type; XY_TWO and XY_FITS read and write interleaved pairs of the
// storage type.
hipError_t launch_xy(int R, int mode, int image_dtype, int storage_dtype, const void *in,
                     void *out, Grid3 g, const Taps &t, const FitArgs *fa, const int *done,
                     hipStream_t s);
hipError_t launch_z_plain(int R, int storage_dtype, const void *in, void *out, Grid3 g,
                          const Taps &t, hipStream_t s);
// Stage-1 z pass: (phi, I) -> the pair (Kz*(H I), Kz*H).
hipError_t launch_z_heaviside(int R, int image_dtype, int storage_dtype, const float *phi,
                              const void *I, void *pair_out, Grid3 g, const Taps &t, float eps,
                              float *probeH, const int *done, hipStream_t s);
// Stage-2 z pass + update from the pair (Kxy*g1, Kxy*g2).
hipError_t launch_z_update(int R, int image_dtype, int storage_dtype, const void *pair_in,
                           Grid3 g, const Taps &t, const UpdArgs &ua, const int *done,
                           hipStream_t s);
hipError_t launch_reduce(const double *partials, int64_t n, double *out, int *flags,
                         double tol_total, hipStream_t s);

// Per-radius, per-type launchers behind the dispatchers (rsf_kernels.hpp).
template <int R, class IT, class ST>
hipError_t launch_xy_r(int mode, const void *in, void *out, Grid3 g, const Taps &t,
                       const FitArgs *fa, const int *done, hipStream_t s);
template <int R, class ST>
hipError_t launch_z_plain_r(const void *in, void *out, Grid3 g, const Taps &t, hipStream_t s);
template <int R, class IT, class ST>
hipError_t launch_z_heaviside_r(const float *phi, const void *I, void *pair_out, Grid3 g,
                                const Taps &t, float eps, float *probeH, const int *done,
                                hipStream_t s);
template <int R, class IT, class ST>
hipError_t launch_z_update_r(const void *pair_in, Grid3 g, const Taps &t, const UpdArgs &ua,
                             const int *done, hipStream_t s);

}  // namespace rsf

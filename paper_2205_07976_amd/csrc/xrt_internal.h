// xrt_internal.h -- structures shared by the host side and the kernels of
// libxrt.  Not part of the public ABI (that is include/xrt.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/xrt.h"

namespace xrt {

// Per-source table row: propagation direction, wavelength, weight, the
// polarization basis (e_perp, dir x e_perp) in which the azimuth psi is
// measured, and 1 / (2 lambda) (the background's sin(theta)/lambda from
// |d - dir|).  12 doubles (96 B), so a row is two aligned scalar loads.
constexpr int SRC_STRIDE = 12;
enum { SRC_DIR = 0, SRC_LAMBDA = 3, SRC_WEIGHT = 4, SRC_E = 5, SRC_B = 8, SRC_HIL = 11 };

// Lower bound of |f| = |h - rint(h)| in the floored form of the sincg lattice
// factor, the form a rotation sum falls back to when one of its terms met
// f = 0 exactly (0/0).  sin^2(pi N f)/sin^2(pi f) = N^2 (1 - (N^2-1) pi^2 f^2
// / 3 + ...), so for |f| <= 2^-32 it equals N^2 to a relative 3.3 N^2 2^-64
// (<= 1.8e-13 at the largest accepted N = 1000, <= 3e-16 at N = 40).
constexpr double F_FLOOR = 2.3283064365386963e-10;  // 2^-32

// Layers of F_default around a structure-factor table.  When the host can
// prove that every rint(h) of a shot lies inside the padded box, the kernels
// index the table without clamping.
constexpr int FHKL_PAD = 8;

struct Params {
    // detector and sample-point geometry (binary64)
    double pixel, distance, beam_f, beam_s;
    double fdet[3], sdet[3], odet[3];
    double layer_dt, atten_len;
    int32_t O, T;
    // regions of interest: n_roi rectangles of roi_nf x roi_ns pixels with
    // origins (i_f, i_s) in `origins`; each is cut into 16 x 16 tiles
    int32_t roi_nf, roi_ns;
    int32_t tiles_f, tiles_per_roi, n_roi, n_tiles;
    // loop extents
    int32_t n_src, n_rot;
    // lattice
    int32_t shape;
    double N[3];
    double gk[3];          // Gaussian: 2 N_i^2 / gauss_c
    double ln_n2;          // Gaussian: log(prod N_i^2)
    double kahn;
    double norm;           // r_e^2 fluence scale / (O^2 n_phi n_mos)
    // structure factors: tables of F^2 with FHKL_PAD layers of F_default^2
    // around the tabulated box.  The element index of entry h0 is
    // h0_a*sa + h0_b*sb + h0_c + zero with sa, sb the strides of the h and k
    // axes and zero the index of h0 = 0; off64 = 2^49 + zero and
    // off32 = 2^50 + zero carry the bias that turns the binary64 sum into the
    // byte offset (see table_offset), for h0 in [lo_d, hi_d].
    const double *F2_64;
    const float *F2_32;
    uint32_t bytes64, bytes32;
    double lo_d[3], hi_d[3];
    double sa, sb;
    double off64, off32;
    // per-shot tables in device memory
    const double *mats;    // [n_rot][9]
    const double *src;     // [n_src][SRC_STRIDE]
    const int32_t *origins;  // [n_roi][2]
    const double *qmats;   // [n_rot][9] rotations umat_m R_k (adjoint only)
    const float *qmats32;  // [n_rot][10] the same in binary32, 9 used (adjoint only)
    double m0[9];          // rows U a_i (adjoint only)
    double m2gk[3];        // -2 gk_i (adjoint only)
    double inv2N[3];       // 2 / N_i (adjoint only)
    // output
    void *image;
    int32_t out_f64;
    int32_t accumulate;
    // split sums: each pixel's outer iterations (sub-pixel, layer, source) in
    // `split` contiguous parts, one workgroup per (tile, part); part sums go
    // to partial[tile][part][lane] and are added in part order afterwards.
    // split == 1: whole sums, no partials.
    int32_t split;
    double *partial;
};

// ---------------------------------------------------------------------------
// Served shots.  A served shot's descriptor and tables live in a pinned host
// arena (written by the host, read by the kernel with range-checked loads, so
// admitting a shot needs no copy on the device); its image lives in the
// device arena, the server's HBM budget.  Work is published as chunks of
// tiles in a ring in pinned host memory.
// ---------------------------------------------------------------------------
constexpr int SERVE_MAX_ROT = 256;   // spindle steps x mosaic domains per served shot
constexpr int SERVE_MAX_SRC = 128;   // sources per served shot
constexpr int SERVE_MAX_CHUNK = 64;  // tiles (or tile parts) per chunk
constexpr int SERVE_MAX_SPLIT = 64;  // parts per pixel sum
constexpr uint32_t SERVE_RING = 1u << 16;  // chunk records and done flags (a power of two)
enum { CHUNK_COMPUTE = 0, CHUNK_REDUCE = 1, CHUNK_BACKGROUND = 2 };

struct ShotDesc {
    Params p;               // pointer fields unused
    uint64_t mats_rel;      // byte offsets of the tables relative to this descriptor
    uint64_t src_rel;
    uint64_t image_off;     // byte offset of the image in the device arena
    uint64_t image_bytes;
    uint64_t partial_off;   // byte offset of the partial sums in the device arena
    uint64_t partial_bytes; // (split > 1 only)
    int32_t roi_f0, roi_s0;
    int32_t clamp;          // 0: every rint(h) of the shot is proven inside the padded table
    int32_t n_seg;          // segments of each unit's outer iterations (>= 1)
    double bg_norm;         // r_e^2 fluence molecules / O^2 of the server's background
    uint64_t state_off;     // byte offset of the running sums between segments
    uint64_t state_bytes;   // (n_seg > 1 only): [unit][lane], 8 bytes each
};

struct ServeChunk {         // written by the host before the tail publishes it
    uint64_t desc_off;      // byte offset of the ShotDesc in the host arena
    int32_t tile0, n_tiles;
    uint32_t seq1;          // chunk number + 1: the value its done flag takes
    uint32_t shot;          // the shot's serial number (nonzero): with desc_off it
                            // names the descriptor a workgroup may keep in LDS
    int32_t kind;           // CHUNK_COMPUTE: units tile * split + part;
                            // CHUNK_REDUCE: tiles whose parts are all done;
                            // CHUNK_BACKGROUND: tiles of a complete image
    int32_t seg;            // CHUNK_COMPUTE: the segment of the units' outer
                            // iterations (every earlier one is done)
};

struct ServeCtrl {          // pinned host memory, written by the host
    uint64_t tail;          // chunks published so far
    uint32_t stop;
    uint32_t pad;
};

struct ServeArgs {
    const ServeCtrl *ctrl;
    const ServeChunk *ring;   // [SERVE_RING], pinned host memory
    uint32_t *done;           // [SERVE_RING], pinned host memory
    unsigned long long *next; // chunks claimed so far (device memory)
    unsigned int *busy;       // workgroups holding a chunk (device memory, 0 at launch)
    unsigned int *exiting;    // set once the kernel is idle: every workgroup leaves
    unsigned long long *last_done;  // s_memrealtime of the latest finished chunk
    const char *hdesc;        // host arena (pinned, coherent)
    uint64_t hdesc_bytes;
    char *arena;              // device arena (images)
    uint64_t arena_bytes;
    const double *F2_64;
    const float *F2_32;
    uint32_t bytes64, bytes32;
    uint64_t idle_ticks;      // 100 MHz ticks of device-wide idleness before the kernel exits
    const void *bg_knots;     // the background's curve records (BgKnot of the server's
                              // precision, device memory), or null: no background
};

// Background of an amorphous scatterer over one region of interest: the
// geometry, sources, image and normalisation of p (n_roi = 1, norm =
// r_e^2 fluence molecules / O^2) and the scattering curve as knots
// (stol_k, F_k, slope_k) with slope_{n-1} = 0, in binary64 and binary32.
constexpr int BG_MAX_KNOTS = 1024;
constexpr int SRC32_STRIDE = 16;
constexpr int SRC32_DIR_LO = 12;
struct BgParams {
    Params p;
    const double *knots64;  // [n_knots][3]
    const float *knots32;   // [n_knots][3]
    const float *src32;     // [n_src][SRC32_STRIDE]: binary32 copies of the source
                            // rows, then dir - (double)(float)dir at SRC32_DIR_LO
    int32_t n_knots;
    int32_t pad;
};

// Launchers (xrt_kernels.hip).  Return the hipError_t of the launch.
// serve_blocks_per_cu: workgroups of the persistent kernel one compute unit
// holds at once (0 on error).
int serve_blocks_per_cu(int precision, int shape);
hipError_t launch_spots(const Params &p, int precision, bool clamp, hipStream_t stream);
hipError_t launch_pad_table(const void *src, int src_f64, int32_t na, int32_t nb, int32_t nc,
                            int32_t pad, double F_default, double *F2_64, float *F2_32,
                            hipStream_t stream);
// Adjoint: partial sums per tile into partial[n_tiles][13], then one
// fixed-order reduction into grad13 that applies the components' constant
// factors (-2 gk_i, 2/N_i and gk_i, inv_scale).
hipError_t launch_grad(const Params &p, int precision, bool clamp, const void *dLdI, int dLdI_f64,
                       double *partial, double *grad13, double inv_scale, hipStream_t stream);
hipError_t launch_serve(const ServeArgs &a, int precision, int shape, int n_wg, hipStream_t stream);
hipError_t launch_sinpi(const double *x, int64_t n, double *s64, float *s32, hipStream_t stream);
hipError_t launch_exp(const double *x, int64_t n, double *y, hipStream_t stream);
hipError_t launch_background(const BgParams &b, int precision, hipStream_t stream);
hipError_t launch_add_image(double *acc, int64_t acc_nf, const void *img, int img_f64, int32_t nf, int32_t ns,
                            int32_t f0, int32_t s0, hipStream_t stream);
// Up to ADD_BATCH whole-accumulator images added in order by one launch (the
// image pointers travel in the kernel arguments).
constexpr int ADD_BATCH = 256;
struct AddBatch {
    const void *img[ADD_BATCH];
};
hipError_t launch_add_images(double *acc, int64_t n_pix, const AddBatch &b, int n_img, int img_f64,
                             hipStream_t stream);
hipError_t launch_trace(const Params &p, int64_t n, const int32_t *idx, double *S, double *h,
                        hipStream_t stream);

}  // namespace xrt

/*
 * xrt.h -- C ABI of the MI355X X-ray tracing library (libxrt.so).
 *
 * The library simulates crystal diffraction images pixel by pixel, as the
 * spots kernel of "Accelerating X-Ray Tracing for Exascale Systems using
 * Kokkos" (section III) does: every pixel of a detector is formed from a
 * physical model of the crystal -- its orientation, its mosaic domains, the
 * photon energy spectrum and one structure factor per Bragg spot (section II,
 * "Scientific background") -- and pixels are independent (section III).
 *
 * For pixel (i_f, i_s) the library computes, in the kinematic model,
 *
 *   I = r_e^2 * fluence * scale / (O^2 * n_phi * n_mos)
 *       * sum_{u,v < O} sum_{t < n_layers}  dOmega * capture_t
 *         * sum_{j < n_src}  w_j * P_j
 *           * sum_{k < n_phi} sum_{m < n_mos}  F(h0)^2 * L^2(h - h0)
 *
 *   sample point  r = Fp fdet + Sp sdet + (distance + t*layer_dt) odet,
 *                 Fp = (i_f + (v + 1/2)/O) pixel - beam_f  (Sp likewise, u)
 *   direction     d = r/|r|; dOmega = pixel^2 (d.odet)/|r|^2
 *   capture_t     exp(-t dt/(mu d.odet)) - exp(-(t+1) dt/(mu d.odet)), or 1
 *                 when layer_dt == 0 (Beer-Lambert)
 *   scattering    S = (d - dir_j)/lambda_j            (1/angstrom)
 *   polarization  P_j = (1 + cos^2 2theta - K cos 2psi sin^2 2theta)/2
 *                 (Kahn et al. 1982; psi measured from the part of evec
 *                 perpendicular to dir_j)
 *   Miller index  h = M_{k,m} S, rows of M_{k,m} = umat_m R(spindle, phi0 +
 *                 k dphi) U {a, b, c}; h0 = nearest integer (ties to even)
 *   lattice       SINCG: prod_i sin^2(pi N_i f_i)/sin^2(pi f_i), f = h - h0
 *                 (limit N_i^2 at f_i = 0); GAUSS: prod_i N_i^2 exp(-2 N_i^2
 *                 f_i^2 / gauss_c)
 *   F(h0)         the table entry, or F_default outside the table.
 *
 * Conventions
 *  - Units: metres (detector), angstrom (wavelengths, cell), radians.
 *  - Arrays are row-major.  Images are [roi_s1-roi_s0][roi_f1-roi_f0], the
 *    fast index contiguous.
 *  - Every call returns an xrt_status: 0 on success, a negative code
 *    otherwise; xrt_last_error() then holds a message (per thread).
 *  - Validation errors are returned before anything is enqueued.  A device
 *    fault is reported as XRT_EDEVICE by the call that sees it.
 *  - Work is enqueued on the caller's HIP stream (a hipStream_t passed as
 *    void*; NULL is the default stream) and is complete when that stream is.
 *  - Every struct starts with struct_size = sizeof(struct); a smaller value
 *    from an older caller is rejected with XRT_EVERSION.
 *  - Host arrays named in a struct (sources, mosaic rotations) are read
 *    during the call only; the caller may free them when it returns.
 *  - Device pointers (structure-factor values, images) stay owned by the
 *    caller and must stay valid until the stream reaches the work.
 *  - No C++ exception crosses this interface.
 */
#ifndef XRT_H
#define XRT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define XRT_VERSION_MAJOR 1
#define XRT_VERSION_MINOR 0

typedef int32_t xrt_status;
enum {
    XRT_OK = 0,
    XRT_EINVAL = -1,   /* an argument is malformed (NaN, negative size, ...) */
    XRT_ERANGE = -2,   /* a size exceeds what the library supports */
    XRT_ENOMEM = -3,   /* a device or host allocation failed */
    XRT_EDEVICE = -4,  /* the HIP runtime reported an error */
    XRT_EBUSY = -5,    /* the object is in use */
    XRT_EVERSION = -6  /* struct_size does not match this library */
};

enum { XRT_SHAPE_SINCG = 0, XRT_SHAPE_GAUSS = 1 };

/* Arithmetic of the sum.
 * XRT_FP64:  every step in IEEE binary64.
 * XRT_MIXED: sample-point geometry, S, h and the reduced arguments f and
 *            N f - rint(N f) in binary64; lattice factor, structure factor and
 *            products in binary32; per-pixel sums compensated (Kahan) in
 *            binary32. */
enum { XRT_FP64 = 0, XRT_MIXED = 1 };

enum { XRT_F32 = 0, XRT_F64 = 1 };

typedef struct xrt_detector {
    uint32_t struct_size;
    int32_t n_fast, n_slow;        /* detector size, pixels (>= 1) */
    double pixel;                  /* pixel pitch, m (> 0) */
    double distance;               /* sample to front face along odet, m (> 0) */
    double beam_f, beam_s;         /* m, along fdet and sdet from the outer corner
                                      of pixel (0, 0) to the foot of the
                                      perpendicular from the sample onto the
                                      detector (Fp = Sp = 0; the direct-beam
                                      spot when the beam runs along odet) */
    double fdet[3], sdet[3], odet[3]; /* fast, slow axes and normal (unit) */
    int32_t oversample;            /* O >= 1 sub-pixels per axis */
    int32_t n_layers;              /* sensor layers >= 1 */
    double layer_dt;               /* layer thickness, m (>= 0; 0 => n_layers 1) */
    double atten_len;              /* attenuation length mu, m (> 0) */
    int32_t roi_f0, roi_f1, roi_s0, roi_s1; /* half-open region of interest */
} xrt_detector;

typedef struct xrt_beam {
    uint32_t struct_size;
    int32_t n_src;                 /* sources >= 1 */
    const double *dir;             /* host [n_src][3] unit propagation directions */
    const double *lambda;          /* host [n_src] wavelengths, angstrom (> 0) */
    const double *weight;          /* host [n_src] weights (finite) */
    double fluence;                /* photons / m^2 */
    double kahn;                   /* polarization factor K */
    double evec[3];                /* polarization direction (unit, not along
                                      any dir_j) */
} xrt_beam;

typedef struct xrt_crystal {
    uint32_t struct_size;
    double cell[9];                /* rows a, b, c in the crystal frame, angstrom */
    double U[9];                   /* orientation (crystal -> lab) */
    int32_t n_mos;                 /* mosaic domains >= 1 */
    const double *umats;           /* host [n_mos][3][3] domain rotations (lab) */
    int32_t n_phi;                 /* spindle steps >= 1 */
    double phi0, dphi;             /* spindle angles, rad */
    double spindle[3];             /* spindle axis (unit) */
    double N[3];                   /* unit cells along a, b, c: SINCG integers in
                                      [1, 1000]; GAUSS reals in (0, 1000] */
    int32_t shape;                 /* XRT_SHAPE_* */
    double gauss_c;                /* Gaussian width constant (> 0) */
    double scale;                  /* overall scale s */
} xrt_crystal;

typedef struct xrt_fhkl_desc {
    uint32_t struct_size;
    int32_t hkl_min[3];            /* first tabulated h, k, l (|.| <= 2^20) */
    int32_t hkl_count[3];          /* entries per axis, >= 1, product < 2^28 */
    int32_t dtype;                 /* XRT_F32 or XRT_F64: type of the values */
    double F_default;              /* structure factor outside the table */
} xrt_fhkl_desc;

/* Opaque structure-factor table resident on one device. */
typedef struct xrt_fhkl xrt_fhkl;

/* Library version (XRT_VERSION_MAJOR / MINOR of the built library). */
xrt_status xrt_version(int32_t *major, int32_t *minor);

/* Message of the last failing call on this thread ("" if none). */
const char *xrt_last_error(void);

/* Structure factors of a crystal (section II: one real structure factor per
 * Bragg spot), made resident on the current device.
 *  dev_F   device pointer to hkl_count[0]*hkl_count[1]*hkl_count[2] values of
 *          type desc->dtype, l fastest.  Read on `stream` before the call
 *          returns (the call synchronises the stream); the caller keeps it.
 *  out     receives a handle owning a padded copy of F^2 in binary64 and
 *          binary32; free it with xrt_fhkl_destroy.
 * Errors: EINVAL (NULL pointers, bad dtype, NaN default), ERANGE (sizes),
 *         ENOMEM, EDEVICE. */
xrt_status xrt_fhkl_create(const xrt_fhkl_desc *desc, const void *dev_F, void *stream,
                           xrt_fhkl **out);

/* Release a table.  The caller must make sure no enqueued work still uses it
 * (synchronise the streams it was used on).  NULL is accepted. */
xrt_status xrt_fhkl_destroy(xrt_fhkl *fhkl);

/* Simulate the region of interest of one shot (section III, the spots
 * kernel: crystal orientation, mosaicity and photon energy).
 *  precision   XRT_FP64 or XRT_MIXED.
 *  dev_image   device pointer, [roi rows][roi cols] of out_dtype.
 *  accumulate  0: the image is overwritten; 1: the new values are added to it
 *              in out_dtype (the separate add-image kernel of section III,
 *              fused into the store).
 * The call uploads a few small tables (cell matrices, sources) stream-ordered
 * and launches one kernel on `stream` (two for split sums, below).
 * Summation order: when the region has fewer than 2048 tiles of 16 x 16
 * pixels, each pixel's loop over (sub-pixel, layer, source) is cut into K
 * contiguous parts summed by different workgroups and the K part sums are
 * added in part order.  K is a function of the shot alone (tile count and
 * loop extents), so a shot's image does not depend on where or beside what it
 * runs.
 * Errors: EINVAL / ERANGE on any malformed field, ENOMEM, EDEVICE. */
xrt_status xrt_simulate(const xrt_detector *det, const xrt_beam *beam,
                        const xrt_crystal *xtal, const xrt_fhkl *fhkl,
                        int32_t precision, void *dev_image, int32_t out_dtype,
                        int32_t accumulate, void *stream);

/* xrt_simulate for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, validation, kernels and bits as xrt_simulate; instead of
 * taking device memory stream-ordered for the shot's tables and the split
 * sums' partial sums, the call uses a static device array of
 * XRT_NOALLOC_SCRATCH_BYTES that every device the library runs on holds
 * until the process ends (tables in its first MiB, partial sums after them).
 * It calls no device allocator (no hipMalloc, hipMallocAsync, hipFree or
 * hipFreeAsync); the tables are copied into the array on `stream`.
 * The array is shared by every call on a device and keeps the last call's
 * contents: calls that overlap on one device (different streams, or other
 * threads) race and must be serialised by the caller; calls one after
 * another on one stream are ordered.
 * Errors: as xrt_simulate; ERANGE when the shot's tables exceed 1 MiB
 * (9 n_phi n_mos + 12 n_src + 1 doubles) or the device ordinal is >= 64. */
#define XRT_NOALLOC_SCRATCH_BYTES ((1u << 20) + (8u << 20))
xrt_status xrt_simulate_noalloc(const xrt_detector *det, const xrt_beam *beam,
                                const xrt_crystal *xtal, const xrt_fhkl *fhkl,
                                int32_t precision, void *dev_image, int32_t out_dtype,
                                int32_t accumulate, void *stream);

/* Simulate n_roi regions of interest of one shot, all roi_nf x roi_ns pixels,
 * in one launch (the per-crystal refinement of section II works on the
 * pixels around predicted Bragg spots).
 *  host_origins  [n_roi][2] int32 (i_f, i_s) of each region's first pixel;
 *                every region must lie inside the detector (det's own ROI
 *                fields are ignored).  Read during the call.
 *  dev_images    device pointer, [n_roi][roi_ns][roi_nf] of out_dtype,
 *                overwritten.
 * Summation order as xrt_simulate, with the tile count of all regions.
 * Errors: as xrt_simulate; ERANGE for n_roi outside [1, 2^22]. */
xrt_status xrt_simulate_rois(const xrt_detector *det, const xrt_beam *beam,
                             const xrt_crystal *xtal, const xrt_fhkl *fhkl,
                             int32_t precision, int64_t n_roi,
                             const int32_t *host_origins, int32_t roi_nf,
                             int32_t roi_ns, void *dev_images, int32_t out_dtype,
                             void *stream);

/* Adjoint of xrt_simulate_rois for the Gaussian shape (refinement of the
 * per-crystal parameters against measured images, section II).  Given
 * dev_dLdI = dL/dI for every pixel of the regions ([n_roi][roi_ns][roi_nf]
 * of dLdI_dtype, device), writes 13 binary64 values to dev_grad13 (device):
 *   [0..8]   dL/dM0, M0 = the 3 x 3 matrix whose rows are U a, U b, U c
 *            (row-major), the cell in the lab frame before spindle and
 *            mosaic rotations;
 *   [9..11]  dL/dNa, dL/dNb, dL/dNc;
 *   [12]     dL/dscale.
 * The sums are reduced in a fixed order (repeat calls give identical bits).
 * Scratch memory for the per-workgroup partial sums is taken stream-ordered.
 * Errors: EINVAL for the sincg shape or scale == 0, otherwise as
 * xrt_simulate_rois. */
xrt_status xrt_backward_rois(const xrt_detector *det, const xrt_beam *beam,
                             const xrt_crystal *xtal, const xrt_fhkl *fhkl,
                             int32_t precision, int64_t n_roi,
                             const int32_t *host_origins, int32_t roi_nf,
                             int32_t roi_ns, const void *dev_dLdI,
                             int32_t dLdI_dtype, double *dev_grad13, void *stream);

/* Background of an amorphous scatterer around the crystal (section III's
 * second kernel, which adds the scattering of the air and the water around
 * the crystal).  The paper gives no formula; the library computes, for every
 * pixel of the detector's region of interest,
 *
 *   I_bg = r_e^2 * fluence * molecules / O^2
 *          * sum_{u,v < O} sum_{t < n_layers}  dOmega * capture_t
 *            * sum_{j < n_src}  w_j * P_j * F_bg(|S_j| / 2)^2
 *
 * with the sample points, S, P_j, dOmega and capture_t of xrt_simulate and
 * F_bg the piecewise-linear interpolant of the curve's knots (constant below
 * the first and above the last).  |S|/2 = sin(theta)/lambda.  The scatterer
 * has no orientation: no spindle or mosaic average. */
typedef struct xrt_background {
    uint32_t struct_size;
    int32_t n_knots;               /* knots of the scattering curve, [2, 1024] */
    const double *stol;            /* host [n_knots] sin(theta)/lambda, 1/angstrom,
                                      finite, strictly increasing */
    const double *F;               /* host [n_knots] scattering factor of one
                                      molecule (finite; every knot and slope
                                      must also be finite in binary32) */
    double molecules;              /* scattering molecules in the beam (>= 0) */
} xrt_background;

/* Background over the detector's region of interest, one kernel on `stream`.
 *  precision   XRT_FP64: every step in binary64.  XRT_MIXED: sample-point
 *              geometry in binary64; d - dir_j from binary32 heads and tails
 *              of d and dir_j (exact where they nearly cancel, next to the
 *              direct beam); |S|/2, the curve, P_j and the products in
 *              binary32; per-pixel sums compensated (Kahan) in binary32.
 *  dev_image   device pointer, [roi rows][roi cols] of out_dtype.
 *  accumulate  0: overwrite; 1: add to the image (a background on top of
 *              xrt_simulate's spots, or several scatterers one after another).
 * The curve and the sources are copied stream-ordered; host arrays are read
 * during the call only.
 * Errors: EINVAL / ERANGE / EVERSION on any malformed field, ENOMEM, EDEVICE. */
xrt_status xrt_simulate_background(const xrt_detector *det, const xrt_beam *beam,
                                   const xrt_background *bg, int32_t precision,
                                   void *dev_image, int32_t out_dtype, int32_t accumulate,
                                   void *stream);

/* Ensemble sum: add a region image into a binary64 accumulator (section III's
 * third kernel adds the results of the other two into one binary64 image; the
 * paper's runs then reduce the images of many shots).  For every pixel (c, r)
 * of the image, acc[s0 + r][f0 + c] += (double) img[r][c].
 *  dev_acc     device, [acc_ns][acc_nf] binary64, updated in place.
 *  dev_img     device, [img_ns][img_nf] of img_dtype (XRT_F32 or XRT_F64),
 *              e.g. a served shot's image read in place.
 *  f0, s0      where the image's first pixel lands; the image must lie inside
 *              the accumulator.
 * One kernel on `stream`; calls on one stream add in call order, so an
 * ensemble summed in a fixed order gives the same bits every time.  The
 * image and the accumulator must not overlap.
 * Errors: EINVAL (NULL, dtype, sizes, placement), ERANGE, EDEVICE. */
xrt_status xrt_add_image(double *dev_acc, int32_t acc_nf, int32_t acc_ns, const void *dev_img,
                         int32_t img_dtype, int32_t img_nf, int32_t img_ns, int32_t f0, int32_t s0,
                         void *stream);

/* Ensemble sum of many whole images: for k = 0 .. n_img-1 in order,
 * acc += (double) img_k, every image [acc_ns][acc_nf] of img_dtype.  The
 * same bits as n_img calls of xrt_add_image in that order; one pass over the
 * accumulator per 256 images instead of one per image.
 *  host_dev_imgs  host array of n_img device pointers, read during the call.
 * Enqueued on `stream`; images must not overlap the accumulator.
 * Errors: EINVAL (NULL, dtype, sizes), ERANGE (n_img outside [0, 2^24]),
 * EDEVICE. */
xrt_status xrt_add_images(double *dev_acc, int32_t acc_nf, int32_t acc_ns,
                          const void *const *host_dev_imgs, int32_t img_dtype, int64_t n_img,
                          void *stream);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of independent shots on one device.
 *
 * The paper runs many simulations per GPU and lets several producers share a
 * GPU to hide latency (section IV, ranks per GPU).  A server owns one arena of
 * device memory (its HBM budget, holding the images and, for shots whose
 * per-pixel sums are split or run in segments, their part sums and running
 * sums) and borrows the structure
 * factors (shared by every shot); shot descriptors and tables sit in pinned
 * host memory that the kernel reads directly.  Submitted shots wait in
 * arrival order; a shot is admitted when its footprint fits in the arena and
 * a resident slot is free; the work of admitted shots is fed in chunks, in
 * the order of the server's policy (below), to a persistent kernel that keeps
 * running while new shots join.  Every pixel is computed exactly
 * as by xrt_simulate with the server's precision (the same summation order),
 * so a shot's image is bit-identical whatever else runs beside it.
 * Calls on one server are serialised internally; progress is driven by
 * xrt_server_progress (call it often: it admits, publishes, launches and
 * collects).  Limits per served shot: n_phi*n_mos <= 256, n_src <= 128.
 *
 * Write-out (host_budget > 0; the paper hides file I/O behind computation by
 * running several producers per GPU, section IV): a shot that finishes on the
 * device is copied into the server's pinned host memory on a copy stream
 * while the persistent kernel goes on with other shots; when the copy is
 * complete the shot's device memory and resident slot are freed and the shot
 * is reported done, and its image is read with xrt_server_host_image.  Device
 * memory thus never waits for a client that is still writing images out;
 * host memory does (finished shots are copied in finishing order as host
 * space frees up, each release making room).
 *
 * Background (desc.background): once a shot's spots are complete, the
 * persistent kernel adds the server's scatterer to its image, in the server's
 * precision, as xrt_simulate_background with accumulate would.
 * --------------------------------------------------------------------------- */
typedef struct xrt_server xrt_server;

typedef struct xrt_server_desc {
    uint32_t struct_size;
    uint64_t hbm_budget;    /* arena bytes, in [1 MiB, 1 TiB] */
    int32_t max_resident;   /* shots admitted at once, in [1, 65536] */
    int32_t precision;      /* XRT_FP64 or XRT_MIXED */
    int32_t shape;          /* XRT_SHAPE_* of every served shot */
    int32_t out_dtype;      /* XRT_F32 or XRT_F64 images */
    int32_t workgroups;     /* persistent workgroups, in [0, 65536]; 0 = as
                               many as the device holds at once less eight,
                               which leaves room for small kernels beside it */
    double idle_exit_us;    /* once no workgroup has work and no chunk has
                               finished for this long, the kernel exits, in
                               [1, 1e6] us; the next progress call relaunches */
    uint64_t host_budget;   /* pinned host bytes for written-out images: 0
                               (images read in place from the device arena)
                               or in [1 MiB, 1 TiB] */
    const xrt_background *background; /* NULL, or a scatterer whose background
                               every served image receives once its spots are
                               complete (the image of xrt_simulate followed by
                               xrt_simulate_background with accumulate, bit
                               for bit); read during xrt_server_create only */
    int32_t policy;         /* XRT_SERVE_FAIR_SHARE or XRT_SERVE_SHORTEST_REMAINING */
    int64_t segment_terms;  /* pixel-terms of a 16 x 16 tile's sums (or of one
                               part of split sums) that one chunk carries at
                               most: a heavier tile's sums run as consecutive
                               segments of its outer iterations, each picking
                               up the running sums the previous one left, so a
                               chunk never holds a workgroup much longer than
                               this and a shot that arrives meanwhile waits
                               less for one; the images keep their bits.  0 =
                               the default 2^21 (a few ms of one workgroup),
                               else in [2^10, 2^40].  Segments need 8 bytes of
                               the device arena per pixel (per part) of a
                               segmented shot. */
} xrt_server_desc;

enum { XRT_SHOT_QUEUED = 0, XRT_SHOT_RUNNING = 1, XRT_SHOT_DONE = 2 };

/* Order in which the work of admitted shots goes to the device.
 * XRT_SERVE_FAIR_SHARE: the next chunk comes from the shot with the least
 *   work (pixel-terms) published so far, a shot admitted later joining at the
 *   current level: resident shots share the device evenly by work
 *   (start-time fair queuing).
 * XRT_SERVE_SHORTEST_REMAINING: the next chunk comes from the shot with the
 *   least work left to publish (shortest remaining processing time): a small
 *   shot overtakes the large ones in flight, which minimises mean latency and
 *   slowdown; under sustained overload the largest shots wait longest.
 * Admission stays in arrival order either way. */
enum { XRT_SERVE_FAIR_SHARE = 0, XRT_SERVE_SHORTEST_REMAINING = 1 };

typedef struct xrt_shot_info {
    uint32_t struct_size;
    int32_t state;          /* XRT_SHOT_* */
    uint64_t image_bytes;
    int32_t roi_nf, roi_ns; /* image is [roi_ns][roi_nf] */
    double t_submit;        /* seconds since the server was created */
    double t_admit;         /* -1 until admitted */
    double t_done;          /* -1 until a progress call has seen it finish */
} xrt_shot_info;

/* Create a server on the current device; fhkl must outlive it.
 * Errors: EINVAL/ERANGE/EVERSION on the descriptor, ENOMEM, EDEVICE. */
xrt_status xrt_server_create(const xrt_server_desc *desc, const xrt_fhkl *fhkl,
                             xrt_server **out);

/* Stop the persistent kernel (it finishes its current chunks), wait for it and
 * free everything; images of unreleased shots become invalid.  NULL is
 * accepted. */
xrt_status xrt_server_destroy(xrt_server *srv);

/* Validate and queue one shot (the detector's ROI); copies every host array,
 * never blocks.  ERANGE if the shot exceeds the served limits or can never
 * fit the budgets. */
xrt_status xrt_server_submit(xrt_server *srv, const xrt_detector *det,
                             const xrt_beam *beam, const xrt_crystal *xtal,
                             uint64_t *ticket);

/* Collect finished work, admit queued shots, publish chunks and (re)launch the
 * persistent kernel if it is not running; *n_done receives the number of
 * shots seen finishing during this call (may be NULL).  The device is kept
 * fed for about a millisecond ahead (every workgroup busy plus half a
 * standard chunk of work per workgroup waiting; a segment's successor is
 * published only once this call has seen it finish), so a request loop that
 * calls it less often than that leaves workgroups idle.  Errors: EINVAL
 * (wrong device), EDEVICE (the kernel or a launch failed). */
xrt_status xrt_server_progress(xrt_server *srv, int32_t *n_done);

/* State and times of a shot.  info->struct_size must be set. */
xrt_status xrt_server_info(xrt_server *srv, uint64_t ticket, xrt_shot_info *info);

/* Device pointer of a finished shot's image inside the arena, valid until
 * xrt_server_release.  EBUSY if not done; EINVAL on a server that writes
 * images out. */
xrt_status xrt_server_image(xrt_server *srv, uint64_t ticket, const void **dev_image);

/* Write-out servers: pointer to a finished shot's image in the server's
 * pinned host memory ([roi_ns][roi_nf] of out_dtype), valid until
 * xrt_server_release.  EBUSY if not done (the copy may still run); EINVAL on
 * a server without a host budget. */
xrt_status xrt_server_host_image(xrt_server *srv, uint64_t ticket, const void **host_image);

/* Free a finished shot's memory and slot (write-out: its host memory; the
 * device memory and the slot were freed when the copy completed).  EBUSY if
 * not done.  The caller must have completed every read of the image first
 * (a copy enqueued on another stream included: synchronise it): the freed
 * region goes to the next admitted shot, whose pixels the running persistent
 * kernel may write at once. */
xrt_status xrt_server_release(xrt_server *srv, uint64_t ticket);

/* Withdraw a shot that is still queued (not yet admitted): the ticket is
 * forgotten and the shots behind it move up.  EBUSY once the shot has been
 * admitted (its work may be on the device: wait for it and release it) or is
 * done; EINVAL for an unknown ticket. */
xrt_status xrt_server_cancel(xrt_server *srv, uint64_t ticket);

/* Diagnostics: the kernels' sin(pi x) for |x| <= 1/2 (the reduced arguments f
 * and g of the lattice factor, section II's crystal-size transform), exactly
 * as the binary64 kernel (dev_s64) and the mixed kernel (dev_s32, from
 * (float)x) form it: x * P(x^2) with P a relative-minimax polynomial.
 * dev_x: [n] binary64; outputs [n]; either output may be NULL, not both.
 * Enqueued on `stream`; outside [-1/2, 1/2] the value is the polynomial's.
 * Errors: ERANGE (n < 0), EINVAL (NULL arrays), EDEVICE. */
xrt_status xrt_sinpi(const double *dev_x, int64_t n, double *dev_s64, float *dev_s32, void *stream);

/* Diagnostics: the binary64 kernels' exp(x) (the Gaussian lattice factor,
 * section II's crystal-size transform in its Gaussian form): reduction by
 * x = (64 k + j) ln2/64 + r, a polynomial for exp(r), the product with a
 * table entry 2^(j/64), scaling by 2^k; for x <= 709.
 * dev_x, dev_y: [n] binary64.  Enqueued on `stream`.
 * Errors: ERANGE (n < 0), EINVAL (NULL arrays), EDEVICE. */
xrt_status xrt_exp(const double *dev_x, int64_t n, double *dev_y, void *stream);

/* Diagnostics: the library's lab-frame cell matrices M_{k,m} (host output,
 * [n_phi*n_mos][3][3], rows a', b', c'), exactly as the kernels receive them. */
xrt_status xrt_cell_mats(const xrt_crystal *xtal, double *host_out);

/* Diagnostics: S and h of n single terms, computed on the device by the same
 * code as the binary64 kernel.  host_idx: [n][6] int32 sextuples (i_f, i_s,
 * u*O + v, t, j, k*n_mos + m); host_S, host_h: [n][3] binary64 outputs.
 * Synchronous (the call waits for the device).
 * Errors: EINVAL/ERANGE on malformed shots or indices, ENOMEM, EDEVICE. */
xrt_status xrt_trace_terms(const xrt_detector *det, const xrt_beam *beam,
                           const xrt_crystal *xtal, int64_t n,
                           const int32_t *host_idx, double *host_S, double *host_h);

#ifdef __cplusplus
}
#endif
#endif /* XRT_H */

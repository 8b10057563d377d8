// xrt_host.h -- host-side helpers shared by the translation units of libxrt
// (validation, error reporting, shot planning).  Not part of the public ABI.
#pragma once

#include <vector>

#include "../../include/xrt.h"
#include "xrt_internal.h"

namespace xrt {
namespace host {

// Record a message for xrt_last_error() and return `code`.
xrt_status fail(xrt_status code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
xrt_status hip_fail(hipError_t e, const char *what);

// Validate a detector (including its ROI), a beam and a crystal.
xrt_status check_shot(const xrt_detector *det, const xrt_beam *beam, const xrt_crystal *xtal);

// Kernel parameters of a one-ROI shot (the detector's ROI) and its tables
// [cell matrices (9 n_rot) | sources (SRC_STRIDE n_src)], as xrt_simulate
// builds them; pointer fields of d->p are not set.
xrt_status served_descriptor(const xrt_detector *det, const xrt_beam *beam, const xrt_crystal *xtal,
                             const xrt_fhkl *fhkl, int32_t out_dtype, ShotDesc *d, std::vector<double> &tables);

// Split factor of a validated one-ROI shot's per-pixel sums (the rule
// xrt_simulate applies; 1 = whole sums).
int32_t split_of(const xrt_detector *det, const xrt_beam *beam, const xrt_crystal *xtal);

// Background of an amorphous scatterer: validation; the curve as rows
// (stol_k, F_k, slope_k; slope 0 at the last knot) in binary64 and their
// binary32 copies ([n][3] each, as the kernels stage them); the
// normalisation r_e^2 fluence molecules / O^2 of a validated shot.
xrt_status check_background_desc(const xrt_background *bg);
void background_rows(const xrt_background *bg, double *k64, float *k32);
double background_norm(const xrt_detector *det, const xrt_beam *beam, double molecules);

// Device tables of a structure-factor handle.
void fhkl_tables(const xrt_fhkl *t, const double **F2_64, const float **F2_32, uint32_t *bytes64,
                 uint32_t *bytes32);

}  // namespace host
}  // namespace xrt

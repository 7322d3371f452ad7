// Width encoding of the bundles (Section 3.4): launchers of render.hip.
#pragma once

#include "hb_internal.h"

namespace hb {

// Density of its edge's layer at every point of the polylines (samples, off_s of desc[0]):
// bilinear in the FP32 density map, negative values as 0, into dens[N]; the largest value, as
// the bits of a non-negative float, into *maxbits (which must start at 0).
hipError_t launch_point_density(const GDesc *desc, const Shape &tot, float *dens, uint32_t *maxbits,
                                hipStream_t st);
// widths[i] = w_min + (w_max - w_min) f(dens[i]) / f(max), f the identity or log1p.
hipError_t launch_widths(const float *dens, int64_t n, const uint32_t *maxbits, double w_min,
                         double w_max, int log_scale, float *widths, hipStream_t st);

}  // namespace hb

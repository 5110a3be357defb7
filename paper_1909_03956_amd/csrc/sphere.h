// Frames (section 3.4, Eq. 18) and the nested equal-area sphere pixelisation
// (section 3.2) of the host runtime.  Extended precision throughout; values
// leave as FP64 after one rounding.
#pragma once

#include <cstdint>

namespace swv {

using ld = long double;

// R_uvw->xyz = R_y(alpha_P) R_x(-delta_P): xyz has y to the celestial pole,
// x to RA 6h, z to RA 0h; uvw has w to the phase centre, u east, v north.
struct Frame {
    ld R[3][3];
};

Frame make_frame(double ra_p, double dec_p);

// SIN projection [l, m, sqrt(1 - l^2 - m^2)] rotated to xyz.
void lm_to_xyz(const Frame& F, double l, double m, ld xyz[3]);

// Level-j nested pixel of an xyz unit vector (1 <= j <= 29).
int64_t ang2pix(int j, const ld xyz[3]);

// Centre of a level-j nested pixel as an xyz unit vector.
void pix2xyz(int j, int64_t pix, ld xyz[3]);

// xyz -> uvw, returned as FP64 (l, m, n - 1).
void xyz_to_lmn(const Frame& F, const ld xyz[3], double* l, double* m, double* nm1);

// N_j = 12 * 4^(j-1) and A_j = 4 pi / N_j.
int64_t n_pixels(int j);
double pixel_area(int j);
// sqrt(A_j) / 4, formed as sqrt(A_1)/4 * 2^(1-j) (equal to the direct
// evaluation, since A_j = A_1 4^(1-j) exactly in binary floating point).
double level_scale(int j);

}  // namespace swv

// Clean loop host helpers (sections 2.1, 3.5).
#pragma once

#include <cstdint>

#include "common.h"

namespace swv {

// Level-J sphere pixel of every pixel of an (nx, ny) image grid with its phase
// centre at (nx / 2, ny / 2); SWV_EDOMAIN if a direction is off the unit disk.
int cross_reference(int J, double ra_p, double dec_p, int nx, int ny, double cell, int64_t* pix);

// Least-squares Gaussian fit of the beam's main lobe: abc = (a, b, c) of
// exp(-(a dx^2 + 2 b dx dy + c dy^2)).
int fit_clean_beam(int nbx, int nby, const double* beam, double abc[3]);

}  // namespace swv

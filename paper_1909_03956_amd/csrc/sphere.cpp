// Nested equal-area pixelisation of the sphere (section 3.2: twelve base
// pixels, four equal-area children per level, N_j = 12 * 4^(j-1)), in the
// HEALPix NESTED layout (Gorski et al. 2005) at nside = 2^(j-1).
//
// Geometry used (the HEALPix projection):
//   * equatorial zone |z| <= 2/3, z = cos(theta):  X = phi / (pi/2), Y = 3z/4;
//   * polar caps: sigma = sqrt(3 (1 - |z|)), X = Xc + (phi/(pi/2) - Xc) sigma
//     with Xc the centre of phi's quarter turn, Y = +-(1 - sigma/2).
// In the (X, Y) plane each base pixel is a square rotated 45 degrees.  With
// A = X + Y + 1/2 and B = Y + 1/2 - X (coordinates along its edges), the
// pair (floor A, floor B) names the base pixel -- floor A + floor B is 1 in
// the north row, 0 in the equatorial row, -1 in the south row -- and the
// fractional parts times nside are the in-face indices (ix, iy), ix growing
// to the north-east, iy to the north-west.  The nested index is
// face * nside^2 + (ix bits at even positions | iy bits at odd positions), so
// the parent of k is k >> 2 (section 3.5).
#include "sphere.h"

#include <cmath>

namespace swv {

static const ld kPi = 3.141592653589793238462643383279502884L;

int64_t n_pixels(int j) { return 12LL << (2 * (j - 1)); }

double pixel_area(int j) { return 4.0 * M_PI / (double)n_pixels(j); }

double level_scale(int j) { return std::ldexp(std::sqrt(pixel_area(1)) / 4.0, 1 - j); }

Frame make_frame(double ra_p, double dec_p) {
    const ld ca = cosl((ld)ra_p), sa = sinl((ld)ra_p);
    const ld cd = cosl((ld)dec_p), sd = sinl((ld)dec_p);
    // R_y(a) = [[ca, 0, sa], [0, 1, 0], [-sa, 0, ca]]
    // R_x(-d) = [[1, 0, 0], [0, cd, sd], [0, -sd, cd]]
    Frame F;
    F.R[0][0] = ca;  F.R[0][1] = -sa * sd;  F.R[0][2] = sa * cd;
    F.R[1][0] = 0;   F.R[1][1] = cd;        F.R[1][2] = sd;
    F.R[2][0] = -sa; F.R[2][1] = -ca * sd;  F.R[2][2] = ca * cd;
    return F;
}

void lm_to_xyz(const Frame& F, double l, double m, ld xyz[3]) {
    const ld L = l, M = m;
    const ld N = sqrtl(1 - L * L - M * M);
    for (int i = 0; i < 3; ++i) xyz[i] = F.R[i][0] * L + F.R[i][1] * M + F.R[i][2] * N;
}

void xyz_to_lmn(const Frame& F, const ld xyz[3], double* l, double* m, double* nm1) {
    ld s[3];
    for (int i = 0; i < 3; ++i) s[i] = F.R[0][i] * xyz[0] + F.R[1][i] * xyz[1] + F.R[2][i] * xyz[2];
    *l = (double)s[0];
    *m = (double)s[1];
    // n - 1 without cancellation on the near hemisphere
    *nm1 = (double)(s[2] > 0 ? -(s[0] * s[0] + s[1] * s[1]) / (1 + fabsl(s[2])) : s[2] - 1);
}

static int64_t spread_bits(int64_t x, int bits, int shift) {
    int64_t out = 0;
    for (int b = 0; b < bits; ++b) out |= ((x >> b) & 1) << (2 * b + shift);
    return out;
}

static int64_t gather_bits(int64_t p, int bits, int shift) {
    int64_t out = 0;
    for (int b = 0; b < bits; ++b) out |= ((p >> (2 * b + shift)) & 1) << b;
    return out;
}

static int64_t floor_div(int64_t a, int64_t b) {
    int64_t q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
    return q;
}

static int mod4(int64_t a) { return (int)(((a % 4) + 4) % 4); }

int64_t ang2pix(int j, const ld xyz[3]) {
    const int64_t nside = 1LL << (j - 1);
    const ld ns = (ld)nside;
    const ld x = xyz[0], z = xyz[1], zx = xyz[2];
    const ld s2 = x * x + zx * zx;  // sin^2(theta)
    ld phi = atan2l(x, zx);
    if (phi < 0) phi += 2 * kPi;
    ld tt = phi / (kPi / 2);
    if (tt >= 4) tt -= 4;
    const ld az = fabsl(z);

    int64_t face, ix, iy;
    if (az > 2.0L / 3.0L) {
        // polar cap; 1 - |z| = sin^2(theta) / (1 + |z|)
        const ld sig = sqrtl(3 * s2 / (1 + az));
        int64_t f = (int64_t)floorl(tt);
        if (f > 3) f = 3;
        const ld tp = tt - (ld)f;
        ld a, b;
        if (z > 0) {
            a = 1 - sig * (1 - tp);
            b = 1 - sig * tp;
            face = f;
        } else {
            a = sig * tp;
            b = sig * (1 - tp);
            face = 8 + f;
        }
        ix = (int64_t)floorl(ns * a);
        iy = (int64_t)floorl(ns * b);
        ix = ix < 0 ? 0 : (ix > nside - 1 ? nside - 1 : ix);
        iy = iy < 0 ? 0 : (iy > nside - 1 ? nside - 1 : iy);
    } else {
        const ld A = tt + 0.75L * z + 0.5L;
        const ld B = 0.75L * z + 0.5L - tt;
        const int64_t Na = (int64_t)floorl(ns * A);
        const int64_t Nb = (int64_t)floorl(ns * B);
        const int64_t p = floor_div(Na, nside), q = floor_div(Nb, nside);
        ix = Na - p * nside;
        iy = Nb - q * nside;
        const int64_t row = p + q;
        face = row == 0 ? 4 + mod4(p) : (row > 0 ? mod4(p - 1) : 8 + mod4(p));
    }
    return face * nside * nside + spread_bits(ix, j - 1, 0) + spread_bits(iy, j - 1, 1);
}

void pix2xyz(int j, int64_t pix, ld xyz[3]) {
    const int64_t nside = 1LL << (j - 1);
    const int64_t face = pix / (nside * nside);
    const int64_t in = pix % (nside * nside);
    const int64_t ix = gather_bits(in, j - 1, 0), iy = gather_bits(in, j - 1, 1);
    const ld a = ((ld)ix + 0.5L) / (ld)nside;
    const ld b = ((ld)iy + 0.5L) / (ld)nside;
    const ld f = (ld)(face % 4);
    const int64_t row = face / 4;  // 0 north, 1 equatorial, 2 south
    ld X, Y;
    if (row == 1) {
        X = (a - b) / 2 + f;
        Y = (a + b - 1) / 2;
    } else {
        X = (a - b) / 2 + f + 0.5L;
        Y = row == 0 ? (a + b) / 2 : (a + b - 2) / 2;
    }
    ld z, st, tt;
    if (fabsl(Y) > 0.5L) {
        const ld sig = Y > 0 ? 2 - (a + b) : a + b;
        const ld omz = sig * sig / 3;  // 1 - |z|
        z = Y > 0 ? 1 - omz : -(1 - omz);
        st = sqrtl(omz * (2 - omz));
        tt = f + 0.5L + (a - b) / (2 * sig);
    } else {
        z = 4 * Y / 3;
        st = sqrtl((1 - z) * (1 + z));
        tt = X;
    }
    const ld phi = tt * (kPi / 2);
    xyz[0] = st * sinl(phi);
    xyz[1] = z;
    xyz[2] = st * cosl(phi);
}

}  // namespace swv

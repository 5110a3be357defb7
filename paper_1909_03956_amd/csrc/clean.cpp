// Host side of the clean loop: the cross-reference table between image pixels
// and level-J sphere pixels (section 3.5) and the clean-beam fit (section 2.1,
// third step).
#include "clean.h"

#include <cmath>
#include <cstring>
#include <deque>
#include <vector>

#include "sphere.h"

namespace swv {

int cross_reference(int J, double ra_p, double dec_p, int nx, int ny, double cell, int64_t* pix) {
    const Frame F = make_frame(ra_p, dec_p);
    const int cx = nx / 2, cy = ny / 2;
    for (int iy = 0; iy < ny; ++iy)
        for (int ix = 0; ix < nx; ++ix) {
            const double l = (double)(ix - cx) * cell, m = (double)(iy - cy) * cell;
            if (!(l * l + m * m < 1.0))
                return fail(SWV_EDOMAIN, "cross reference: pixel (%d, %d) is off the unit disk",
                            ix, iy);
            ld xyz[3];
            lm_to_xyz(F, l, m, xyz);
            pix[(int64_t)iy * nx + ix] = ang2pix(J, xyz);
        }
    return SWV_OK;
}

int fit_clean_beam(int nbx, int nby, const double* beam, double abc[3]) {
    const int cx = nbx / 2, cy = nby / 2;
    const auto at = [&](int y, int x) { return beam[(int64_t)y * nbx + x]; };
    if (!(at(cy, cx) >= 0.5)) return fail(SWV_EDOMAIN, "clean beam: beam centre below 1/2");
    // main lobe: 8-connected pixels >= 1/2 reachable from the centre
    std::vector<unsigned char> seen((size_t)nbx * nby, 0);
    std::deque<std::pair<int, int>> todo;
    seen[(size_t)cy * nbx + cx] = 1;
    todo.emplace_back(cy, cx);
    // normal equations of  -ln B = a dx^2 + 2 b dx dy + c dy^2  over the lobe
    double M[3][3] = {}, r[3] = {};
    int64_t count = 0;
    while (!todo.empty()) {
        const auto [y, x] = todo.front();
        todo.pop_front();
        const double dx = x - cx, dy = y - cy;
        const double row[3] = {dx * dx, 2.0 * dx * dy, dy * dy};
        const double rhs = -std::log(at(y, x));
        for (int i = 0; i < 3; ++i) {
            for (int k = 0; k < 3; ++k) M[i][k] += row[i] * row[k];
            r[i] += row[i] * rhs;
        }
        ++count;
        for (int ddy = -1; ddy <= 1; ++ddy)
            for (int ddx = -1; ddx <= 1; ++ddx) {
                const int yy = y + ddy, xx = x + ddx;
                if (yy < 0 || yy >= nby || xx < 0 || xx >= nbx) continue;
                unsigned char& s = seen[(size_t)yy * nbx + xx];
                if (!s && at(yy, xx) >= 0.5) {
                    s = 1;
                    todo.emplace_back(yy, xx);
                }
            }
    }
    // Cholesky of the 3 x 3 normal matrix; a lobe that does not determine the
    // three parameters leaves a pivot at rounding level
    double Lc[3][3] = {};
    const double scale = M[0][0] + M[1][1] + M[2][2];
    for (int i = 0; i < 3; ++i) {
        for (int k = 0; k <= i; ++k) {
            double s = M[i][k];
            for (int q = 0; q < k; ++q) s -= Lc[i][q] * Lc[k][q];
            if (i == k) {
                if (!(s > 1e-10 * scale))
                    return fail(SWV_EDOMAIN,
                                "clean beam: the %lld-pixel main lobe does not determine the fit",
                                (long long)count);
                Lc[i][i] = std::sqrt(s);
            } else {
                Lc[i][k] = s / Lc[k][k];
            }
        }
    }
    double z[3], x[3];
    for (int i = 0; i < 3; ++i) {
        double s = r[i];
        for (int q = 0; q < i; ++q) s -= Lc[i][q] * z[q];
        z[i] = s / Lc[i][i];
    }
    for (int i = 2; i >= 0; --i) {
        double s = z[i];
        for (int q = i + 1; q < 3; ++q) s -= Lc[q][i] * x[q];
        x[i] = s / Lc[i][i];
    }
    if (!(x[0] > 0 && x[2] > 0 && x[0] * x[2] - x[1] * x[1] > 0))
        return fail(SWV_EDOMAIN, "clean beam: the fit is not a peaked Gaussian");
    std::memcpy(abc, x, sizeof x);
    return SWV_OK;
}

}  // namespace swv

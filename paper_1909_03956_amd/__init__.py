"""Model-visibility prediction on MI355X (gfx950): the direct component sum and
the spherical-Haar-wavelet tree of Skipper, Scaife & McEwen (2019), with the
exact adjoint and chi^2 gradients, behind the C ABI of libswvis.so
(include/swvis.h).  This package only marshals torch tensors into that
library; the library must be built (build.py) -- there is no CPU fallback.
"""
from ._lib import SwvError, lib  # noqa: F401
from .api import (BatchPlan, Context, Graph, MajorCycle, Tree, adjoint, ang2pix, context,  # noqa: F401
                  cross_reference, dirty_beam, dirty_image, fit_clean_beam, grad_direct, hogbom,
                  image_grid, pixel_centres, pixels_in_disk, predict_degrid, predict_direct,
                  residual_chi2,
                  restore, synchronize, wavelet_clean)

from . import autograd  # noqa: F401,E402

__version__ = "1.0"

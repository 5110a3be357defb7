"""Seeded synthetic inputs shared by the GPU path's tests/bench and the oracle.

Input manufacture only (array layouts, Earth-rotation tracks, component
models, noise); it contains none of the method's arithmetic and imports
neither the oracle nor the GPU package.  The paper's measurement sets are
not available, so these tracks stand in for its JVLA-style simulations.
"""
from . import configs, models, tracks  # noqa: F401

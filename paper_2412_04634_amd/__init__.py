"""MI355X-native neural incident radiance cache (NIRC) and two-level Monte Carlo estimator.

``nirc`` is the ctypes binding of the HIP library (include/nirc.h); ``workload`` draws the seeded
synthetic inputs (shading points, lobe field, initial weights).
"""
from . import workload  # noqa: F401

"""RT-CDF sort for AMD Instinct MI355X (gfx950).

``paper_2609_00843_amd.rtcdf`` is the binding of the HIP library (loaded on
import, fails loudly if it is not built); ``paper_2609_00843_amd.inputs`` holds
the seeded synthetic workloads.  Importing the package itself loads nothing.
"""

__all__ = ["rtcdf", "inputs"]

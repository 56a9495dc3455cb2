"""MI355X-native sampling estimator for influence minimization by node blocking.

The compute path lives in the HIP library ``libimin.so`` (C ABI in
``include/imin.h``); :mod:`paper_2405_12871_amd.binding` marshals arguments
to it.  :mod:`paper_2405_12871_amd.synth` draws seeded synthetic inputs.
Importing the package loads nothing native.
"""

__all__ = ["binding", "synth", "build"]

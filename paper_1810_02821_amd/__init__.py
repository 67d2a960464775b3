"""Messenger-field Wiener filter and Wiener-posterior sampler for AMD MI355X.

The library (libmf.so, C ABI in include/mf.h) runs Algorithm 1 of Jeffrey,
Heavens & Fortio, "Fast Sampling from Wiener Posteriors for Image Data with
Dataflow Engines" as hand-written HIP kernels for gfx950.  This package is its
thin Python face:

* ``Plan``      - problems and device tables (``mf_plan_create``);
* ``Schedule``  - cooling schedule of the Wiener filter;
* ``Plan.wiener / sample / wiener_backward / band_power`` - the entry points;
* ``autograd.WienerFilter`` - a torch.autograd.Function over the Wiener map;
* ``synth``     - seeded synthetic workloads (no method arithmetic).
"""
from ._binding import (Info, MFError, NotConverged, Plan, Schedule, lib)  # noqa: F401


def __getattr__(name):
    # torch-dependent helpers load lazily
    if name == "autograd":
        import importlib
        return importlib.import_module(".autograd", __name__)
    raise AttributeError(name)

__all__ = ["Plan", "Schedule", "Info", "MFError", "NotConverged", "lib"]

"""Seeded synthetic inputs shared by the HIP path's tests and benchmark and by the oracle.

This package draws random numbers and lays out arrays; it computes nothing of the
flow-matching method itself (no network, no integrator, no sampling noise). Both the
HIP path and the FP64 oracle consume what it produces:

* ``events``   truth particle sets (CSR offsets + 9-feature rows), multiplicity laws
                of the benchmark configurations;
* ``params``   the flat FP32 parameter vector of the stand-in velocity network, in the
                canonical order both sides unpack independently;
* ``configs``  the named model/workload configurations;
* ``arrivals`` Poisson request streams for the serving form;
* ``errors``   the error measures used to compare any two outputs (normwise per
                feature, response mean/width).

The paper (Sec. 2.2) describes the neural backend as a conditional flow-matching model
sampled by Euler integration, conditioned on the truth particles of each event; it fixes
no architecture, feature encoding or dataset that is available here, so everything in
this package is a synthetic stand-in with the laws stated in each module.
"""

from . import configs, events, params, arrivals, errors  # noqa: F401

"""FP64 CPU oracle of conditional flow-matching sampling — TEST INFRASTRUCTURE ONLY.

This package is the checker, not the product. Only the test suite, the smoke check of
the entry module and the CPU-baseline leg of the benchmark may import it. The HIP path
never imports, links or calls it, and it shares no code with the HIP path: the two meet
only through the seeded inputs of the ``workload`` package.

What it computes (the paper, Sec. 2.2 and Sec. 1): the neural detector backend is a
continuous-time generative model trained with conditional flow matching, conditioned on
the truth-level particles of each event, and sampled by integrating its learned vector
field from noise with Euler steps whose number is set at run time. The paper fixes no
network, time grid or noise law; the stand-in network and the readings used for every
silent point are stated in each module. Everything is plain NumPy float64, one event at
a time, with no padding, batching, caching, fusion or reordering.

Modules:
  philox     Philox4x64-10 counter-based generator and the Box-Muller noise law
  net        unpacking of the flat parameters; LayerNorm, GELU, Linear, attention;
             truth encoder; time embedding; the velocity field
  ode        explicit Euler and classic RK4 on a uniform grid
  observables  H_T, MET and lepton isolation of reconstructed events (Sec. 2.4)
  sample     per-event sampling driver and output decoding
  select     truth preprocessing: model pT cut and particle limit

Pins (tests marked "not gpu"): Philox against the generator of NumPy and the published
known-answer vector; Box-Muller moments; LayerNorm, GELU and softmax textbook
identities; attention special cases and brute force on tiny sets; the closed-form
product solution of a linear field for Euler and RK4; Euler/RK4 convergence orders on
the real network; slot-permutation equivariance and truth-permutation invariance;
reduction identities of the network under zeroed weights.
"""

from .philox import philox4x64_10, uniforms23, noise_event, noise_batch  # noqa: F401
from .net import (unpack, layer_norm, gelu, linear, attention, softmax_rows,  # noqa: F401
                  time_features, encode_truth, velocity)
from .ode import integrate, stage_times  # noqa: F401
from .sample import simulate, simulate_events, decode  # noqa: F401

"""FP64 CPU oracle for the MPS sampling sweep.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The HIP sampler shares
no code with it (no kernels, headers, helpers or tables); the only thing both
sides consume is the seeded input generator, which holds none of the
sampling arithmetic.

* ``philox``  -- Philox4x64-10 and the FP64 uniform per (seed, chain, sample, site).
* ``sampler`` -- the sequential sampler (Section 2.2; Section 3.3.1, Algorithm 1),
  its forced-prefix mode, the optional per-sample displacement of the
  physical index (Section 3.4.1, Eq. 7), the direct amplitude product and
  brute-force enumeration used to pin it.

Every function is pinned by a CPU test (closed forms, invariants, brute force,
a library cross-check); none is "parity unpinned".
"""
from .philox import philox4x64, philox4x64_np, uniforms, bits_to_uniform  # noqa: F401
from .sampler import sample, forced_probs, draw, amplitude_norm2, brute_force, config_index, displacement  # noqa: F401

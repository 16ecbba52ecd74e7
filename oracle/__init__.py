"""Plain, slow FP64 CPU oracle of the road-surface stereo path.

TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import, call or execute anything here.  The HIP library and
its Python binding never do, and the two share no code: no kernels, helpers,
tables or constants.  The only module both sides read is ``synth`` (seeded inputs,
no arithmetic of the method).

  oracle.stereo   forward path (warp, ZNCC volumes, bilateral aggregation, WTA,
                  left-right check, parabola subpixel, post-processing, 3-D points)
  oracle.adjoint  loss of the differentiable form and its exact gradient
  oracle.restricted  restricted-search aggregation (Sec. IV): windows around the
                  unaggregated WTA, windowed WTA, the rest of the full path
  oracle.plane    road-plane estimation (Sec. II-A): RANSAC over given draws,
                  least-squares refit, roll angle

Pins (tests marked "not gpu") tie every function to facts fixed by the paper or
by mathematics rather than to itself; see tests/test_oracle_*.py.
"""
from . import stereo, adjoint, restricted, plane  # noqa: F401

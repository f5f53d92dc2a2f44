"""FP64 CPU oracle for the NeuralVDB coordinate-MLP encode/decode.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
package: only the tests, the smoke check and the CPU-baseline leg of the
benchmark use it.  It shares no code with the HIP library; the two meet only
through seeded inputs produced by the ``workloads`` package.

Every function is written from the paper (NeuralVDB, arXiv 2208.04448) in
plain numpy, float64 for all floating point, with no blocking or fusion.
Where the paper leaves a detail open, the reading taken is stated in the
function's docstring.

Modules
  tree     -- VDB [Hash,5,4,3] build and coordinate decomposition (Sec. 3.1)
  mlp      -- feature mapping (eq. fm), MLP, losses (eq. mse, BCE, CE),
              hand-derived backward, Adam and the learning-rate staircase
  sampler  -- counter-based SplitMix64 batch indices
  fit      -- training loop, full decode and error report
  moe      -- sparse domain decomposition: subdomains, tent gates, blended
              decode (eq. moe)
"""
from . import tree, mlp, sampler, fit, moe  # noqa: F401

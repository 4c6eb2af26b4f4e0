"""Plain FP64 CPU oracle of the 3DGS^2-TR optimizer iteration.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this
package.  It shares no code with the HIP path: the only common dependency is
the seeded input generator in ``synthetic/``, which holds none of the method's
arithmetic.

Layout (each module cites the paper passages it follows):

* ``gaussians`` -- the Gaussian primitive, its parameterisation and SH colour
  (Background, Eq. gaussian-primitive).
* ``binning``   -- projection, tile keys, stable sort and per-tile ranges,
  emulated op-for-op in IEEE float32 so keys are comparable bit for bit.
* ``render``    -- FP64 projection and front-to-back alpha blending (Background,
  the blending equation), differentiable with torch autograd.
* ``loss``      -- the per-pixel L1 / D-SSIM loss split into components
  (Eq. pixel_loss) and the least-squares objective (Eq. objective).
* ``method``    -- stochastic gradient, Gauss-Newton HVP, Hutchinson estimate,
  squared Hellinger distance, the trust-region radius SHD, the TR step of
  Algorithm 1, Algorithm 1 as a plain loop over t (``run_tr``), the Adam
  baseline, the epsilon schedule and PSNR.

Parity status of each function is listed in its docstring; every function has
at least one pin in ``tests/test_oracle_*.py`` except those marked
"parity unpinned".
"""

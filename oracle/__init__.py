"""Plain FP64 CPU oracle of the sparse-pixel Gaussian rasterizer hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
package: only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg
of ``bench.py`` use it.  It shares no code with the HIP library; the only
common module is ``synth`` (seeded inputs, no method arithmetic).

The oracle is written for a reader with the paper at hand: slow, vectorised
with numpy where that keeps the formulas visible, FP64 throughout except where
the method fixes a storage precision (half error map, uint16 age map) or where
a floating-point value decides an integer (the sort key carries the depth as
FP32 bits).  Each function cites the passage it follows.

Modules:
  sh         real spherical-harmonic basis (degree <= 3)
  params     raster / loss / optimizer parameter records
  project    EWA projection + SH colour                    (Sec. 3.1)
  binning    tile x depth keys, sort, per-tile ranges      (Sec. 3.1, 3.6)
  rng        counter-based SplitMix64 draws
  sampler    tile-wise error/age pixel sampling            (Sec. 3.5)
  render     front-to-back compositing and its adjoint     (Eq. alpha_comp, Sec. 3.6)
  loss       Charbonnier L1 + tile sparse NCC              (Sec. 3.7, App. A)
  maps       error-map EMA, age update, dense error init   (Sec. 3.3)
  project_bwd  chain rule from screen space to parameters
  optim      moment-damped LM + Adam                       (Sec. 3.9, App. A)
  pipeline   one training step composed from the above
"""

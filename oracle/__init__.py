"""FP64 CPU oracle of the Instant-NVR rendering back-end hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) imports, calls or links anything in this package; only the test
suite, the smoke check and the bench's ``cpu_baseline`` leg do.

It is a plain, slow, obviously-correct restatement of what the hot path
computes, written in float64 NumPy (pure-Python loops only over tiny
dimensions), following

* the paper's own definitions where it gives them: the dual-quaternion blend
  and its inverse (Sec. 4.1 Eq. 1, Sec. 4.2 Eq. 4), the node influence weight
  exp(-|v - x_i|^2 / r^2) with r = 0.1 (Sec. 4.1), the per-sample look-up of
  neighbouring nodes (Sec. 4.2, "On-the-fly Radiance Fields") and the colour /
  depth supervision (Sec. 4.3, Eq. 8);
* the published definitions of the methods the paper builds on where it
  delegates (Sec. 4.2 and 4.3 build the fields on Instant-NGP and render them
  by NeRF volume rendering): multiresolution hash encoding, tiny density /
  colour networks with a spherical-harmonics view encoding, alpha compositing
  and Adam.

Where the paper is silent the reading taken is stated in each module header.

Modules:
    grid       multiresolution hash encoding, forward + backward
    sh         real spherical harmonics of the view direction
    network    density + colour networks, forward + backward
    composite  volume-rendering compositing, forward + closed-form backward
    march      ray / box clipping and occupancy-skipping sample placement
    warp       hybrid warp (inverse skinning then inverse node blend) + backward
    optim      loss (Eq. 8 reading) and Adam with loss scaling
    step       whole training step and forward-only render
"""
from . import grid, sh, network, composite, march, warp, optim, step  # noqa: F401

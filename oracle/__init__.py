"""Plain, slow FP64 CPU oracle for the SGAD-SLAM splatting hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may call it.  It shares no code with the HIP library; both sides
consume the seeded inputs of ``paper_2603_21055_amd.synth`` and nothing else.

Modules
-------
* ``splat``  – preprocess, contribution rule, brute-force and culled
  compositing, the analytic adjoint and the tile-binning integer function
  (paper Sec. 3.2, "Rendering RGB and Depth by Splatting"; the splat
  operation is defined along the 3DGS lineage the paper builds on).
* ``se3``    – Exp/Log on SE(3) for the left-twist pose parametrisation.
* ``track``  – per-pixel depth-distribution residuals, Jacobians and
  Gauss-Newton (abstract; Sec. 3.3 per-point Gaussian model).
* ``loss``   – L1 photometric/depth terms of Eq. 1 and their upstream grads.
* ``optim``  – Adam step with the paper's learning rates.
* ``conv``   – FP64 3x3 conv net with BF16 rounding emulation.
"""

"""MI355X-native splatting of pixel-aligned Gaussians at adjusted depth.

The compute path is the HIP library ``libsgad.so`` (C ABI, ``include/sgad.h``);
``paper_2603_21055_amd.sgad`` is its thin ctypes binding and
``paper_2603_21055_amd.synth`` generates seeded synthetic inputs.
"""

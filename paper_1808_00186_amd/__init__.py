"""MI355X-native edge-FEM CSEM secondary-field solver (HIP, gfx950).

The compute path lives in the HIP library built from ``csrc/``; ``petgem`` is
its ctypes binding and ``synth`` the seeded workload generator.
"""

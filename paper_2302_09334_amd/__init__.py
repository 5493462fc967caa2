"""MI355X-native fused world step of the non-episodic neuroevolution simulator
of arXiv 2302.09334 (HIP kernels for gfx950 behind a C-ABI library).

``world``     ctypes binding of ``libworld.so`` (torch supplies memory + streams)
``workloads`` seeded synthetic workload definitions
``batch``     many uneven worlds advanced in one launch
``serve``     continuous-batching serving loop
"""
__all__ = ["world", "workloads"]

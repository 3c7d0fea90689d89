"""MI355X-native splat-and-trace path for heat-haze refraction.

SPH particles -> refractive-index excess delta-n = n - 1 on a voxel grid
(Gladstone-Dale) with its central-difference gradient -> curved-ray marching
with the curvature-driven adaptive step -> exit rays and per-pixel
displacement maps.  All compute runs in the HIP library `libhaze.so`
(gfx950); `paper_2603_02048_amd.haze` is its thin Python binding and
`paper_2603_02048_amd.workloads` draws seeded synthetic inputs.
"""

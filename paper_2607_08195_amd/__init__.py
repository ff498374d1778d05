"""MI355X-native DSMC particle loop (move, counting sort, NTC/VHS collisions,
cell moment sampling) behind a C ABI, with a thin Python binding.

The binding lives in ``paper_2607_08195_amd.dsmc``; seeded synthetic inputs
in ``paper_2607_08195_amd.workloads``.
"""

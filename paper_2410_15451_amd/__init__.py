"""Static / ND / DS / DF Leiden community detection on AMD MI355X (gfx950).

The compute path is the HIP library ``libleiden_mi355x.so`` behind the C-ABI
declared in ``include/leiden.h``; ``binding`` marshals arguments to it.
``inputs`` holds the seeded synthetic input generators.
"""

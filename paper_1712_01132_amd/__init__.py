"""poredvm: an MI355X (gfx950) implementation of the iterative discrete-velocity
solve of the steady linearised BGK equation on voxelised porous media
(Ho et al., "A multi-level parallel solver for rarefied gas flows in porous
media", Sec. 2-3).

The compute path is the C-ABI library `libporedvm.so` (HIP kernels for gfx950);
`poredvm` is its thin ctypes binding. Importing this package does not load the
library; `poredvm.Solver` does, and fails loudly if it is missing.
"""

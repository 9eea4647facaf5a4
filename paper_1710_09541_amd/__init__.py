"""MI355X (gfx950) implementation of the phase-field lattice Boltzmann step of Liang et al.
(arXiv:1710.09541): two coupled D2Q9 lattices, conservative Allen-Cahn for the order
parameter and incompressible Navier-Stokes with the paper's forcing distribution.

The compute path is the HIP library ``liblbm_hip.so`` (C-ABI in ``include/lbm.h``);
``paper_1710_09541_amd.lbm`` is its ctypes binding and ``paper_1710_09541_amd.cases``
builds seeded synthetic workloads.
"""

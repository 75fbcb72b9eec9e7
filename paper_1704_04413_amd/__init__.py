"""MI355X-native recursive-regularized lattice Boltzmann step.

The compute path is the HIP library ``librrlbm.so`` (C-ABI, see include/rrlbm.h);
``binding`` marshals arguments to it.  Importing this package loads nothing:
``from paper_1704_04413_amd import binding`` does.
"""

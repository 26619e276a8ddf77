"""Seeded synthetic inputs for the polarization / screened-interaction path.

This package builds input arrays only: lattice, k-mesh, plane-wave spheres,
orthonormal wavefunction coefficients, band energies, frequency grids,
transition probabilities and Wannier orbitals on the real-space grid.  It
holds none of the method's arithmetic (no pair densities, no weights, no
polarization, no dielectric matrix, no projection).  Both the FP64 oracle and
the device library consume exactly these arrays.
"""

from .gen import (  # noqa: F401
    BOHR_ANGSTROM,
    HARTREE_EV,
    Problem,
    at_qpoint,
    make_problem,
    qpoint_gvectors,
    mesh_fractions,
    batch_system,
    batch_system_qpoints,
    parity_workload,
    srvo3_workload,
    supercell_workload,
)

from .symmetric import screw_ops, star_table, symmetric_problem  # noqa: F401,E402

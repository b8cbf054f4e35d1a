"""CPU oracle of the CutFEM vertex-patch multigrid (TEST INFRASTRUCTURE ONLY).

A plain, slow, obviously correct NumPy/SciPy implementation of what the GPU
path computes, written from the paper "A multigrid method for CutFEM and its
implementation on GPU" (Cui, Kanschat): assembled sparse matrices, explicit
prolongation matrices, dense local inverses and a textbook V-cycle and PCG,
all in float64.  It shares no code with the HIP library and must only be
imported by the tests, by the smoke check and by the CPU-baseline leg of the
benchmark.  The product path never calls it.

Modules and the passages they follow:
  basis       Q_k Gauss-Lobatto nodal basis (Section 2.1, eq. (spaces))
  geometry    nested Cartesian levels, active/cut cells, DoFs (Section 2.1, Section 3)
  quadrature  cut-cell rules by dimension reduction (Section 3, substitute quadrature)
  assemble    Nitsche form + face ghost penalty, load vector (eqs. (cutfem_nitsche),
              (cutfem-ghost), (weak-equation))
  transfer    embedding prolongation and its transpose (Section 2.2)
  multigrid   vertex patches, coloured MVS, V-cycle, PCG (Section 2.3, eqs.
              (local-solver), (smoother), (smoother-split); Section 4 set-up)
  problem     builds all of it for a workload

Pins (tests/test_oracle_*.py) tie every part to something other than itself:
the paper's 27 DoF counts, closed-form areas/volumes/moments, exact element
matrices, Nitsche identities on polynomials, hand-computed ghost jumps,
polynomial reproduction of the prolongation, the Kronecker structure of the
patch Laplacian, coloured vs sequential MVS without ghost coupling, the
two-grid formula, V-cycle symmetry, direct solves and O(h^{k+1}) convergence.
Parity unpinned: iteration counts on the benchmark geometries (the paper
reports GMRES counts on a different domain), the choice of the ghost-penalty
exponent, and single-precision results beyond their reported deviation.
"""

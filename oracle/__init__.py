"""Plain FP64 CPU oracle for the DMRG superblock hot path.

TEST INFRASTRUCTURE ONLY. Nothing in the product package imports this
package; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run it.

It is written from the paper (Alvarez, "The Density Matrix Renormalization
Group for Strongly Correlated Electron Systems: A Generic Implementation"),
slow and obvious on purpose, and shares no code with the HIP path:

* ``models``     site operators, Hamiltonians (Sec. 4.1), exact
                 diagonalisation by bit strings (the pins' ground truth).
* ``superblock`` the superblock product y = H psi (Sec. 1, Eq. (1); Sec. 3.3
                 outer product of operators; Sec. 3.3 per-symmetry-block
                 evaluation) as an explicit Kronecker matrix, as dense
                 A Psi B^T and per symmetry block.
* ``lanczos``    lowest eigenpair with full reorthogonalisation (Sec. 3.3).
* ``rho``        reduced density matrices (Eqs. (2)-(3)), their spectra,
                 truncation to m states and the truncation error (Sec. 1).
* ``dmrg``       the infinite loop (Sec. 3.1, Fig. 2) and finite sweeps
                 (Sec. 1), on dense block operators.

Every function names the passage it follows. Where the paper is silent the
reading used is stated in the docstring.
"""

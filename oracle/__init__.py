"""Plain FP64 CPU oracle for mixed real/momentum-space cylinder DMRG.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.  The
product path (the HIP library and its Python binding) never imports it and
shares no code with it.

Modules (each function cites the passage of Motruk, Zaletel, Mong and Pollmann,
"DMRG on a cylinder in mixed real and momentum space", arXiv:1512.03318, that it
follows):

* ``model``       Hofstadter cylinder term lists, real-space basis (eq. H_real) and
                  mixed basis (eqs. H_kin, H_int).
* ``ed``          bitstring exact diagonalisation with Jordan-Wigner signs (eq. JW).
* ``free``        free-fermion closed form from eq. H_kin (finite cylinders and the
                  Bloch bands of the infinite cylinder).
* ``mpo``         finite-state-machine MPO construction (Sec. IV A-D, eq. MPO),
                  trimming and exact deparallelisation, dense contraction.
* ``blocksparse`` U(1) x Z_Ly block-sparse tensors, environment updates and the
                  two-site effective-Hamiltonian matvec (standard DMRG, the paper
                  relies on it without restating it).
* ``lanczos``     host Lanczos with full reorthogonalisation and an FP64
                  tridiagonal eigensolve.
* ``dmrg``        finite two-site DMRG with block-wise SVD truncation.
* ``idmrg``       infinite-cylinder DMRG by unit-cell growth on the bulk MPO cell.
* ``synth``       environments contracted from seeded isometries.
"""

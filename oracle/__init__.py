"""CPU oracle for the two-site TDVP (2TDVP) step -- TEST INFRASTRUCTURE ONLY.

A plain, slow, complex128 NumPy/SciPy implementation of what the HIP path
computes, written from the paper (Xie et al., arXiv 1908.10588):

* hamiltonian  -- local boson / electronic operators and the el-vib
                  Hamiltonian of Section 2.2 (eqs. Hamiltonian, Hel_2,
                  Hvib_2, Helvib_2) as a sparse matrix in the full product
                  space;
* mpo          -- the same Hamiltonian as an MPO (eq. MPO), by a prefix-trie
                  finite-state construction;
* mps          -- product states, canonical forms (eqs. l/r orthonormal),
                  MPS <-> dense vector;
* tdvp         -- environments, effective Hamiltonians (eqs. one-site
                  Hamiltonian 1 and two-site Hamiltonian), Lanczos
                  exponential, DBSS/SVD truncation and the 2TDVP sweep
                  (Section 2.1.2);
* observables  -- populations, norm, energy, autocorrelation C(t) (Sec. 3.1);
* exact        -- exact propagation in the full product space and closed
                  forms used to pin everything above.

Only the tests, the smoke check of the package entry point and the benchmark's
CPU-baseline leg may import this package.  It shares no code with the HIP
library and never imports it.
"""
HBAR = 0.6582119569  # eV * fs

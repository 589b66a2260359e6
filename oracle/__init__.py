"""CPU FP64 oracle for the additive two-level DMRG hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link or
execute anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the
HIP library (no kernels, headers, helpers or table generators); the only common
input is the seeded generator module ``seeded_inputs``.

Contents
--------
``fock``      second-quantised Hamiltonian on the Fock space via Jordan-Wigner
              (Section 3.2), exact diagonalisation in an (N, Sz) sector and the
              one-particle reduced density matrix.
``tt``        tensor-train utilities written from the definitions of Section 2.1
              (contraction map, orthogonal decompositions, retraction operators),
              QN-blocked truncated SVD and LQ, classical two-site DMRG
              (Algorithm 1) and the additive two-level DMRG (Algorithm 2 with the
              subdomain grouping of Extension Two) whose local problems are
              solved from the explicit projected operator ``P^T A P``
              (Lemma "DMRG micro-iterations for eigenvalue problems") and whose
              coarse matrices are formed from dense state vectors
              (eq. A_reduced).  Dense vectors limit it to small L (<= 8).
``contract``  einsum definitions of the environment tensors (eq. env_L, env_R),
              the two-site matvec (eq. mat_vec, two-site form) and the
              gradients of ``<x|H_eff|x>``; used for kernel-level parity at
              any size on sampled outputs.
``lanczos``   a plain Lanczos eigensolver with full reorthogonalisation.
``mpo``       the oracle's own matrix product operator of the Hamiltonian
              (eq. MPO), built from Jordan-Wigner site factors of every term;
              independent of the library's MPO builder.
``chain``     two-site DMRG (Algorithm 1) and the additive two-level DMRG
              (Algorithm 2, Extension Two) through environment chains only:
              Lanczos local solves on the effective operator, coarse matrices
              as TT inner products and sandwiches (Appendix A.2), Step 4 as TT
              rounding of the direct-sum TT.  No dense state vector, so it
              reaches L = 12..16 at chi = 128..160 (minutes to hours).
``density``   one-particle density matrix by transfer matrices.
"""

"""Additive two-level DMRG hot path on AMD MI355X (gfx950).

``api``     Python binding of the C ABI (include/tt.h); the work runs in the HIP
            library ``libtt.so`` built in-tree by ``build``.
``mpo``     host-side construction of the Hamiltonian as a sparse MPO.
"""

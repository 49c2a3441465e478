"""Plain, slow CPU oracle of the iPEPS hot path (TEST INFRASTRUCTURE ONLY).

This package is the correctness reference for the HIP implementation in
``paper_1910_11359_amd``.  It is imported only by ``tests/``, by
``__graft_entry__.smoke()`` (to check one small device run) and by the
``cpu_baseline`` leg of ``bench.py``.  The product path never imports it.

Everything here is complex128 NumPy/SciPy in the natural (ket ⊗ bra) basis,
written step by step after the method section of arXiv:1910.11359
("Setting" → "Set up for iPEPS": initialization, quench with the simple
update, readout with CTMRG) and its appendix (D, δt, d = d_p·d_A, χ ≥ D²).
It shares no code with the device path: no kernels, helpers or tables.

Modules
    model    local space, dilated bond Hamiltonian (Eq. Hanc), Trotter gates
    peps     initial Néel ⊗ |+⟩ state, Trotter layers, plain simple update
    ctmrg    double layer, directional CTMRG with half-system projectors,
             corner-spectrum convergence, one-site reduced density matrix
    run      job schedules (time series of imbalance and occupations)

Parity status per function is listed in each module header.
"""

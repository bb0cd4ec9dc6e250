"""Plain FP64 CPU oracle for TTN-HEOM propagation (TEST INFRASTRUCTURE ONLY).

This package is the slow, obviously-correct reference that the GPU library is
checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it; the product path
(``paper_2603_17711_amd``) never does, and the two share no code.

Everything here is complex128 / float64 NumPy written from the paper
(arXiv 2603.17711, "TENSO"):

* ``bath``        -- bath-correlation features (Sec. II A, Eq. bcfdecores, Eqs. DL, BO)
* ``sop``         -- the sum-of-products generator (Sec. II B, Eqs. heom-std,
                     dissipator, master_lvn) and the dense HEOM reference
* ``ttn``         -- tree tensor networks (Sec. II C, Eqs. omega_tensor, semiunitary),
                     environments, effective generators, reduced density matrix
* ``integrators`` -- RK4 sub-flows and the ps1 / ps2 projector-splitting sweeps
                     (Sec. II C, last two paragraphs)
* ``mlp``         -- FP64 reference MLP for the learned surrogate

Pins (what each function is checked against) are listed in each module
header; a function with no independent pin says "parity unpinned".
"""

"""FP64 CPU oracle for the asynchronous DG method with AT fluxes.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.

Plain, slow, obviously correct NumPy code written from the paper
(Goswami & Aditya, "An asynchronous discontinuous Galerkin method for
massively parallel PDE solvers", arXiv 2404.03399).  Every function cites
the section / equation / table it follows.  It shares no code, tables or
constants with the device library; the only common input is
``paper_2404_03399_amd.workloads`` (problem parameters and seeded draws).

Modules
  basis     reference element: GLL nodes, M, S, K-matrices (Sec. 2, Eq. 7-8)
  atflux    AT-flux coefficients from the moment conditions (Sec. 5, Table 1)
  delays    counter-based delay schedule (Sec. 6.1 delay emulation)
  stepper   DG / ADG / ADG-AT / naive ADG with Heun, SSP-RK3, RK4
  exact     exact solutions (advection; inviscid Burgers by characteristics)
  fourier   Fourier-mode analysis (Sec. 4.2)
  adjoint   reverse-mode discrete adjoint of the stepper
  stats     error norms, conservation integral, ensemble statistics

Parity unpinned: nothing in the forward path; see each module's header.
"""

"""Plain FP64 CPU oracle for the Vanka-star / phMG / FGMRES hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports this
package; only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` may call it.  It shares no code with the GPU path: its
own reference element, quadrature, DoF numbering, assembly, patches, LU,
relaxation, transfers, V-cycle and FGMRES.  Only the seeded meshes and the
analytic problem data come from the shared ``synth`` input package.

Every function cites the passage of the paper it follows:
  * Section 2, eqs. "eq:stokes-eq", "eq:stokes-disc", "eq:saddle" -- problem, weak form, saddle matrix;
  * Section 2.1 -- Taylor-Hood and Scott-Vogelius spaces, quadrisection / Alfeld meshes;
  * Section 3.1, eq. "eq:TG-operator" -- hMG two-level propagator, P = FE interpolation, R = P^T;
  * Section 3.2, eq. "eq:DC-TG-operator" -- phMG defect correction;
  * Section 3.4, eq. "eq:ASM" and figure "fig:patches" -- additive Schwarz Vanka-star patches, exact LU;
  * Section 4 (solver setup paragraph) -- coarse direct solve, restarted FGMRES(30).

Pin status of each function is recorded in its module docstring; there is no
function in this package without a pin in ``tests/test_oracle_*.py``.
"""

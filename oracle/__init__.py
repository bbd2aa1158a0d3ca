"""ORACLE -- test infrastructure, not product code.

A plain, slow, FP64 CPU implementation of the solve phase of the monolithic
defect-correction AMG preconditioner for Stokes (Voronin, MacLachlan, Olson,
Tuminaro, arXiv 2306.06795), written from the paper:

  sa.py      Algorithm 1: per-field smoothed-aggregation hierarchies, block
             interpolation, Galerkin coarse saddle operators (Section 3.2)
  vanka.py   algebraic Vanka patches and additive Vanka with a dense LU solve
             of every full patch matrix (Section 3.3.1)
  dlsc.py    Chebyshev semi-iteration and the DLSC sweep (Algorithm 2,
             Section 3.3.2, Table 2)
  dc.py      the defect-correction cycle, eq. (3.1) with eq. (3.2) and the
             multilevel eq. (3.4); schedules DC-all / DC-skip1 / DC-skip0, and
             HO-AMG (Algorithm 1 applied to K0, the remark after it)
  fgmres.py  restarted, right-preconditioned FGMRES(20) (Section 4)
  sparse.py  structural sparse products, a counter-based generator

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
import it.  It shares no code with the HIP library and imports nothing from it.
"""

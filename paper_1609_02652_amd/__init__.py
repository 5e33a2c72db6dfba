"""PF-MP HMC hot path on MI355X: even-odd Wilson-clover operator, solvers,
polynomial filter, forces and integrator behind the ``libpfmp`` C-ABI.

The HIP library is loaded lazily by :mod:`paper_1609_02652_amd.pfmp`; importing the
package itself (for example for the seeded input generators in ``synth``) touches
no GPU.
"""

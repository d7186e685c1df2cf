"""cps: curvilinear pressure-Poisson multigrid for MI355X (gfx950).

The solver lives in the HIP C-ABI library ``libcps.so`` built from
``csrc/``; ``paper_2305_17875_amd.cps`` is its thin ctypes binding and
``paper_2305_17875_amd.inputs`` the seeded input generators.  Importing the
package loads nothing; the binding loads the library on first use and raises
if it is missing.
"""
__all__ = ["cps", "inputs"]

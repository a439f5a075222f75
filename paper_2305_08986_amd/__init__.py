"""MI355X-native generalized-Stokes hot path (Q2-Q1 matrix-free operator,
monolithic block multigrid, FGMRES) for semi-implicit ALE fluid-structure
interaction.

The compute path lives in the HIP library ``libfsi.so`` built from ``csrc/``;
``paper_2305_08986_amd.fsi`` is its thin ctypes binding.  Importing the
package itself loads nothing.
"""
__all__ = ["fsi", "workloads"]

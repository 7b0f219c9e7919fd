"""MI355X-native time-domain ferroelectric phase-field step (TDGL with
Poisson and hex8-FEM elasticity), after Ashraf & Salahuddin, arXiv:1202.6116.

Importing the package loads nothing native; `paper_1202_6116_amd.pf` is the
binding to the HIP library, `paper_1202_6116_amd.workloads` the problem
descriptions and seeded inputs.
"""
__all__ = ["pf", "workloads"]

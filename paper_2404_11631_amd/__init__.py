"""MI355X-native batched stochastic Frank-Wolfe simulation (Algorithm 1 of He, Liu, Wu, Zheng
and Zhu, Section 3.1) behind a C ABI.

Importing the package loads nothing native; the HIP library is loaded on first use by
``paper_2404_11631_amd.sim`` and raises if it has not been built.
"""
__all__ = ["workloads"]

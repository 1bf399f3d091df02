"""Seeded synthetic inputs shared by the decoder library and its CPU oracle.

Holds code constructions, the space-time workload graph and the fault
sampler.  None of the decoder's arithmetic lives here.
"""
from . import gf2, codes, sampler, workloads  # noqa: F401
from .codes import Problem  # noqa: F401
from .workloads import WORKLOADS, TABLE_I, DecoderParams, problem, shots_for  # noqa: F401

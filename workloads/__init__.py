"""Seeded synthetic inputs shared by the oracle and the HIP library.

This package holds no arithmetic of the ADG method: it only shapes inputs
(initial states, the synthetic reaction mechanism, delay-model parameters and
case sizes).  Both sides receive identical arrays from here.
"""
from .gen import *  # noqa: F401,F403

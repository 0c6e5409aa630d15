"""BDDC-SO (balancing domain decomposition by constraints on subobjects) for
MI355X: the C-ABI HIP library and its thin Python binding."""
from ._binding import BDDCSOError, EXPORTED, LIB_PATH, load  # noqa: F401
from .solver import BDDCSOSolve, Preconditioner, Problem, copy_probe, default_options  # noqa: F401

"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

Holds problem descriptions and workload generators only; none of the
method's arithmetic lives here."""
from .problem import *  # noqa: F401,F403
from . import configs  # noqa: F401

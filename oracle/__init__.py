"""Test infrastructure only: the plain FP64 CPU oracle (see oracle.py).  Never imported by the
product library."""
from .oracle import *  # noqa: F401,F403

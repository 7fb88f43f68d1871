"""Seeded synthetic inputs for the tall-skinny and randomized low-rank SVD.

This package generates test matrices, sketching matrices and cotangents.  It
is shared by the CPU oracle's tests, the GPU parity tests and the benchmark so
that both sides see identical bytes.  It contains no step of the SVD method
itself: no TSQR, no orthonormalization, no small SVD, no sketch products.
"""
from .matrices import *  # noqa: F401,F403

"""Shared helpers of the GPU parity tests (test code, not product code)."""
import math

import numpy as np

U64 = 2.0 ** -53
U32 = 2.0 ** -24


def gamma(n, u):
    """Higham's gamma_n = n u / (1 - n u): bound on the relative rounding
    error of a length-n recursive sum of products."""
    return n * u / (1.0 - n * u)


def square_bound(n, prec):
    """Worst-case |S_gpu - S_ref| for one symmetric square of an iterate with
    spectrum in [0,1] (sum_k |x_ik||x_jk| <= 1 by Cauchy-Schwarz on rows of
    norm <= 1), when both sides round the same inputs but sum in different
    orders: each side is within gamma of the exact sum. bf16x3 sums 3n
    exact products."""
    if prec == "fp64":
        return 2 * gamma(n, U64)
    if prec == "fp32":
        return 2 * gamma(n, U32)
    return 2 * gamma(3 * n, U32)


def print_case(msg):
    print(msg, flush=True)

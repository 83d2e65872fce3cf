"""Shared helpers of the GPU parity tests."""

import functools

import numpy as np

from oracle import sg
from sg_inputs import named_problem


@functools.lru_cache(maxsize=None)
def system(name, **kw):
    prob = named_problem(name, **dict(kw))
    return prob, sg.build_system(prob)


def cached_system(name, **kw):
    return system(name, **kw)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))

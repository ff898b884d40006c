"""Differentiable D0 and D2 persistence of a scalar field on the GPU path.

Forward (Section 2.5, 2.6): GPU order, discrete gradient and critical
simplices; the extremum graph on the GPU (D0: descents from the critical
edges, triplets sorted by edge; D2: ascents on the dual complex from the
critical triangles, triplets by decreasing triangle), the union-find on the
host over the sorted triplets; births and deaths are the highest vertex
values of each simplex (dms_simplex_values).  Backward: the library's
scatter kernel sends dL/d(birth, death) to the max vertices.
"""
import numpy as np


def _torch():
    import torch
    return torch


def _make():
    torch = _torch()
    from . import (critical_simplices, d0_pairs, d2_pairs, dims_of, discrete_gradient, gradient_backward,
                   order, simplex_values)

    def _backward(ctx, g_births, g_deaths):
        birth_code, death_code = ctx.saved_tensors
        gb = (g_births if g_births is not None else torch.zeros(birth_code.numel())).to(
            device=birth_code.device, dtype=torch.float64).contiguous()
        gd = (g_deaths if g_deaths is not None else torch.zeros(death_code.numel())).to(
            device=death_code.device, dtype=torch.float64).contiguous()
        grad = gradient_backward(birth_code, death_code, gb, gd, ctx.n)
        return grad.reshape(ctx.shape)

    def _finish(ctx, field, birth_code, death_code):
        births = simplex_values(field, birth_code).to(field.dtype)
        deaths = simplex_values(field, death_code).to(field.dtype)
        ctx.save_for_backward(birth_code, death_code)
        ctx.n = field.numel()
        ctx.shape = field.shape
        return births, deaths

    class PersistenceD0(torch.autograd.Function):
        """apply(field) -> (births, deaths): float tensors of the finite D0
        pairs, in the order the pairing visits them (increasing death edge)."""

        @staticmethod
        def forward(ctx, field):
            dims = dims_of(field)
            with torch.no_grad():
                o = order(field)
                rec = discrete_gradient(o)
                lists, counts = critical_simplices(rec, dims)
                pe, pm = d0_pairs(rec, o, dims, lists[0], lists[1])
            dev = field.device
            death_code = torch.from_numpy(pe).to(dev)
            birth_code = torch.from_numpy(pm).to(dev) << 8
            return _finish(ctx, field, birth_code, death_code)

        @staticmethod
        def backward(ctx, g_births, g_deaths):
            return _backward(ctx, g_births, g_deaths)

    class PersistenceD2(torch.autograd.Function):
        """apply(field) -> (births, deaths) of the D2 pairs (2-saddle
        triangle, maximum tet), in the order the pairing visits them
        (decreasing birth triangle)."""

        @staticmethod
        def forward(ctx, field):
            dims = dims_of(field)
            with torch.no_grad():
                o = order(field)
                rec = discrete_gradient(o)
                lists, counts = critical_simplices(rec, dims)
                pt, pq = d2_pairs(rec, o, dims, lists[2], lists[3])
            dev = field.device
            birth_code = torch.from_numpy(pt).to(dev)
            death_code = torch.from_numpy(pq).to(dev)
            return _finish(ctx, field, birth_code, death_code)

        @staticmethod
        def backward(ctx, g_births, g_deaths):
            return _backward(ctx, g_births, g_deaths)

    return PersistenceD0, PersistenceD2


_made = []


class _Lazy(object):
    """Builds the autograd.Functions on first use so that importing the
    package does not import torch."""

    def __init__(self, which):
        self._which = which

    def apply(self, *args):
        if not _made:
            _made.extend(_make())
        return _made[self._which].apply(*args)


PersistenceD0 = _Lazy(0)
PersistenceD2 = _Lazy(1)


def d0_loss(births, deaths, threshold=0.05):
    """Sum of squared persistence of the pairs below the threshold."""
    pers = deaths - births
    keep = pers < threshold
    return (pers[keep] ** 2).sum()

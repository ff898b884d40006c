"""Differentiable D0 persistence of a scalar field on the GPU path.

Forward (Section 2.5, 2.6): GPU order, discrete gradient and critical
simplices; the extremum graph (descents from the critical edges, triplets
sorted by edge) on the GPU, Algorithm 1's union-find on the host over the
sorted triplets; births and deaths are gathered from the field as the
highest vertex value of each simplex.  Backward: the
library's scatter kernel sends dL/d(birth, death) to the max vertices.
"""
import numpy as np


def _torch():
    import torch
    return torch


def _make():
    torch = _torch()
    from . import critical_simplices, d0_pairs, discrete_gradient, dims_of, gradient_backward, order

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
            birth_vertex = torch.from_numpy(pm).to(dev)
            birth_code = birth_vertex << 8
            flat = field.reshape(-1)
            births = flat[birth_vertex]
            deaths = flat[death_code >> 8]
            ctx.save_for_backward(birth_code, death_code)
            ctx.n = flat.numel()
            ctx.shape = field.shape
            return births, deaths

        @staticmethod
        def backward(ctx, g_births, g_deaths):
            birth_code, death_code = ctx.saved_tensors
            gb = (g_births if g_births is not None else torch.zeros(birth_code.numel())).to(
                device=birth_code.device, dtype=torch.float64).contiguous()
            gd = (g_deaths if g_deaths is not None else torch.zeros(death_code.numel())).to(
                device=death_code.device, dtype=torch.float64).contiguous()
            grad = gradient_backward(birth_code, death_code, gb, gd, ctx.n)
            return grad.reshape(ctx.shape)

    return PersistenceD0


class _Lazy(object):
    """Builds the autograd.Function on first use so that importing the package
    does not import torch."""

    def __init__(self):
        self._fn = None

    def _get(self):
        if self._fn is None:
            self._fn = _make()
        return self._fn

    def apply(self, *args):
        return self._get().apply(*args)


PersistenceD0 = _Lazy()


def d0_loss(births, deaths, threshold=0.05):
    """Sum of squared persistence of the pairs below the threshold."""
    pers = deaths - births
    keep = pers < threshold
    return (pers[keep] ** 2).sum()

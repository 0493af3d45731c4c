"""torch front end: softened self-gravity as an autograd Function.

``SFGravity.apply(pos, mass, soft, opts_dict)`` returns (acc, pot) computed by
the GPU library (tree path by default, direct path with ``path="direct"``);
its backward calls the library's adjoint on the same handle.  PyTorch only
provides device memory and the stream.
"""
from __future__ import annotations

import torch

from . import _lib


class SFGravity(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos, mass, soft, cfg):
        cfg = dict(cfg or {})
        path = cfg.pop("path", "tree")
        opts = _lib.make_opts(**cfg)
        pos, mass, soft = pos.contiguous(), mass.contiguous(), soft.contiguous()
        if path == "tree":
            tree = _lib.sf_grav_build_tree(pos, mass, soft, opts)
            acc, pot = _lib.sf_grav_accel(tree, None, None, None, opts)
        elif path == "direct":
            tree = None
            acc, pot = _lib.sf_grav_accel(None, pos, mass, soft, opts)
        else:
            raise ValueError(f"unknown path {path!r}")
        ctx.tree = tree
        ctx.opts = opts
        ctx.save_for_backward(pos, mass, soft)
        return acc, pot

    @staticmethod
    def backward(ctx, g_acc, g_pot):
        pos, mass, soft = ctx.saved_tensors
        if g_acc is None:
            g_acc = torch.zeros((pos.shape[0], 3), dtype=pos.dtype, device=pos.device)
        want = tuple(bool(x) for x in ctx.needs_input_grad[:3])
        gx, gm, gh = _lib.sf_grav_accel_backward(ctx.tree, pos, mass, soft, ctx.opts, g_acc,
                                                 g_pot, want=want)
        if ctx.tree is not None:
            _lib.sf_grav_tree_free(ctx.tree)
            ctx.tree = None
        return gx, gm, gh, None


def gravity(pos, mass, soft, **cfg):
    """Accelerations (n,3) and potentials (n,) with autograd support."""
    return SFGravity.apply(pos, mass, soft, cfg)

"""torch front end: softened self-gravity as an autograd Function.

``SFGravity.apply(pos, mass, soft, opts_dict)`` returns (acc, pot) computed by
the GPU library (tree path by default, direct path with ``path="direct"``);
its backward calls the library's adjoint on the same handle.  PyTorch only
provides device memory and the stream.
"""
from __future__ import annotations

import torch
from torch.autograd.function import once_differentiable

from . import _lib


class SFGravity(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos, mass, soft, cfg):
        cfg = dict(cfg or {})
        path = cfg.pop("path", "tree")
        field = cfg.pop("field", None)
        opts = _lib.make_opts(**cfg)
        pos, mass, soft = pos.contiguous(), mass.contiguous(), soft.contiguous()
        if path == "tree":
            tree = _lib.sf_grav_build_tree(pos, mass, soft, opts)
            if field is not None:
                _lib.sf_grav_tree_set_field(tree, field.detach().contiguous())
            acc, pot = _lib.sf_grav_accel(tree, None, None, None, opts)
        elif path == "direct":
            tree = None
            acc, pot = _lib.sf_grav_accel(None, pos, mass, soft, opts)
        else:
            raise ValueError(f"unknown path {path!r}")
        # the handle lives as long as the graph node (Tree frees it when
        # collected), so a second backward (retain_graph=True) walks the same
        # tree with the same decisions
        ctx.path = path
        ctx.tree = tree
        ctx.opts = opts
        ctx.save_for_backward(pos, mass, soft)
        return acc, pot

    @staticmethod
    @once_differentiable
    def backward(ctx, g_acc, g_pot):
        pos, mass, soft = ctx.saved_tensors
        if ctx.path == "tree" and (ctx.tree is None or not ctx.tree.handle):
            raise RuntimeError("SFGravity: the tree handle of this graph was freed")
        if g_acc is None:
            g_acc = torch.zeros((pos.shape[0], 3), dtype=pos.dtype, device=pos.device)
        want = tuple(bool(x) for x in ctx.needs_input_grad[:3])
        gx, gm, gh = _lib.sf_grav_accel_backward(ctx.tree, pos, mass, soft, ctx.opts, g_acc,
                                                 g_pot, want=want)
        return gx, gm, gh, None


def gravity(pos, mass, soft, **cfg):
    """Accelerations (n,3) and potentials (n,) with autograd support.

    cfg: the sf_grav_opts fields of ``make_opts`` (form, theta, order, alpha,
    ...), ``path`` ("tree" or "direct") and, for alpha >= 0 on the tree path,
    ``field``: the previous accelerations (n, 3) for the relative criterion.
    """
    return SFGravity.apply(pos, mass, soft, cfg)

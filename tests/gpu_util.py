"""Helpers shared by the GPU tests (tensor conversion, handle creation)."""
import numpy as np
import torch

from paper_2006_12883_amd import stmg


def dev():
    return torch.device("cuda:0")


def T(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).to(dev())


def H(prob, **opt):
    return stmg.Handle(prob, device="cuda:0", **opt)


def rel_err(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def assert_close(got, ref, rtol, what=""):
    """Max-norm comparison scaled by max(1, |ref|_max), with a short message."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    assert got.shape == ref.shape, (what, got.shape, ref.shape)
    scale = max(1.0, float(np.abs(ref).max()) if ref.size else 1.0)
    err = float(np.abs(got - ref).max()) if ref.size else 0.0
    if not err <= rtol * scale:
        idx = np.unravel_index(int(np.argmax(np.abs(got - ref))), ref.shape)
        raise AssertionError("%s: max err %.3e > %.1e * %.3e at %s (got %.6e, ref %.6e)"
                             % (what, err, rtol, scale, idx, got[idx], ref[idx]))

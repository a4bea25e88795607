"""Shared helpers of the GPU parity tests (not collected by pytest)."""
import numpy as np

TIE_EPS = 2.0 ** -44


def device_problem(p):
    """Copy a workloads.Problem to CUDA tensors (same bytes as the oracle sees)."""
    import torch
    d = {"b": torch.from_numpy(np.ascontiguousarray(p.b)).cuda()}
    if p.fmt == "dense":
        d["A"] = torch.from_numpy(np.ascontiguousarray(p.A)).cuda()
    else:
        d["values"] = torch.from_numpy(np.ascontiguousarray(p.values)).cuda()
        d["row_ptr"] = torch.from_numpy(np.ascontiguousarray(p.row_ptr, dtype=np.int64)).cuda()
        d["col_idx"] = torch.from_numpy(np.ascontiguousarray(p.col_idx, dtype=np.int32)).cuda()
    return d


def make_solver(p, dev=None, **kw):
    from paper_1806_02968_amd import Solver
    dev = dev or device_problem(p)
    if p.fmt == "dense":
        return Solver(dev["A"], dev["b"], **kw), dev
    return Solver(values=dev["values"], row_ptr=dev["row_ptr"], col_idx=dev["col_idx"], shape=(p.m, p.n),
                  b=dev["b"], **kw), dev


def compare_samples(o_idx, o_gap, g_idx, g_gap, eps=TIE_EPS):
    """Drawn indices must agree wherever neither side is within the tie band."""
    clear = (o_gap > eps) & (g_gap > eps)
    mism = np.nonzero(o_idx[clear] != g_idx[clear])[0]
    ties = int((~clear).sum())
    return mism.size, ties


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))

"""Helpers of the GPU tests: move a workloads.Graph and blocks to the device."""
import numpy as np
import torch

import paper_1509_08863_amd as asc

DEV = "cuda:0"


def to_dev(x, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(DEV)


def upload_graph(g, w=None, unit_as_null=False, validate=False):
    rp = to_dev(g.row_ptr.astype(np.int32))
    ci = to_dev(g.col_idx.astype(np.int32))
    if w is None and not unit_as_null:
        w = g.weights_or_ones()
    wt = None if w is None else to_dev(np.asarray(w, dtype=np.float32))
    return asc.graph_prepare(rp, ci, wt, validate=validate)


def block_f32(x, ld=None):
    """float32 device block with leading dimension ld (>= r, multiple of 4)."""
    x = np.asarray(x, dtype=np.float32)
    n, r = x.shape
    ld = ld or (r + 3) // 4 * 4
    buf = torch.zeros(n, ld, dtype=torch.float32, device=DEV)
    buf[:, :r] = torch.from_numpy(x).to(DEV)
    return buf[:, :r]


def block_bf16(bits, ld=None):
    """bfloat16 device block from bf16 bit patterns (uint16)."""
    bits = np.asarray(bits, dtype=np.uint16)
    n, r = bits.shape
    ld = ld or (r + 7) // 8 * 8
    buf = torch.zeros(n, ld, dtype=torch.bfloat16, device=DEV)
    buf[:, :r] = torch.from_numpy(bits.view(np.int16)).to(DEV).view(torch.bfloat16)
    return buf[:, :r]


def scalar(x):
    return torch.tensor([float(x)], dtype=torch.float64, device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_fro(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))

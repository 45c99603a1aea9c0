"""Shared helpers of the GPU tests: the library context, operators built from
the seeded generators, and the oracle runs they are compared against."""
import functools
import sys

import numpy as np

import synth


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@functools.lru_cache(None)
def torch_mod():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    return torch


@functools.lru_cache(None)
def ctx():
    from paper_0707_0502_amd import gdr
    torch = torch_mod()
    return gdr.gdr_ctx_create(0, torch.cuda.current_stream().cuda_stream)


def dev(a):
    torch = torch_mod()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).cuda()


def host(t):
    torch_mod().cuda.synchronize()
    return t.cpu().numpy()


def empty(n):
    torch = torch_mod()
    return torch.zeros(n, dtype=torch.complex128, device="cuda")


def make_op(links, kappa, bc=(1, 1, 1, -1), link_storage=1):
    from paper_0707_0502_amd import gdr
    lt, lz, ly, lx = links.shape[1:5]
    return gdr.gdr_wilson_create(ctx(), (lx, ly, lz, lt), bc, kappa, np.ascontiguousarray(links),
                                 link_storage)


@functools.lru_cache(None)
def config_data(name):
    cfg = synth.CONFIGS[name]
    links = synth.gauge_links(cfg["dims"], cfg["eps"], cfg["seed"])
    B = np.stack([synth.make_rhs(cfg, k, s).ravel() for k, s in cfg["rhs"]])
    return cfg, links, synth.kappa(name), B


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)

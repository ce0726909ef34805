"""Helpers shared by the GPU tests: the library binding, seeded inputs moved to
the device, and results moved back for comparison with the CPU oracle."""
import numpy as np


def rp():
    import paper_2304_04612_amd as m
    return m


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def bits16(t):
    """int16 tensor of FP16 patterns -> uint16 numpy array."""
    return host(t).view(np.uint16)


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)

"""Shared helpers of the GPU parity tests: build the oracle problem and the
HIP plan from one configuration, move fields between numpy and torch."""
import numpy as np

from oracle.pipe import Pipe
from oracle import optimize as opt
from paper_2509_10103_amd import synth


def make(cfg):
    P = Pipe(cfg["nr"], cfg["nt"], cfg["nz"], cfg["lz"], cfg["re"], cfg["wo"], cfg["amp"], cfg["dt"], cfg.get("t0", 0.0))
    from paper_2509_10103_amd import npo
    G = npo.Plan(cfg["nr"], cfg["nt"], cfg["nz"], cfg["lz"], cfg["re"], cfg["wo"], cfg["amp"], cfg["dt"],
                 cfg.get("t0", 0.0), cfg.get("nsteps", 1))
    return P, G


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def seed_field(P, seed, e0):
    """Oracle-projected, normalised smooth solenoidal perturbation."""
    return opt.normalise(P, opt.project(P, synth.solenoidal_modes(P.r, P.M, P.K, P.lz, seed)), e0)


def relerr(P, a, b):
    """||a - b||_W / ||b||_W."""
    d = a - b
    return np.sqrt(P.wdot(d, d) / P.wdot(b, b))


def maxrel(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))

"""Writes fd_config5.json: FP64 central finite differences of the lattice
divergence (the oracle's) for images 0 and 1 of the 1024 x 1024 gray batch
(M = 256, sigma = 4): dD/dh over the 32 x 32 crop u, v in [496, 528) and
dD/dw for codevectors 0..31, with h = 1e-4.

Calls only the oracle and the seeded input generators. Usage:
    python tests/golden/make_fd_config5.py
"""
import json
import multiprocessing as mp
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_1310_7114_amd import synth as S  # noqa: E402

H_FD = 1e-4
CROP = (496, 528)
NW = 32
_CASE = {}


def _D(I, W, sigma, R):
    return O.lattice_divergence(I, (O.density_map(I, sigma, R),), W, sigma)


def _pixel(args):
    u, v = args
    c = _CASE
    Ip = c["I"].copy(); Ip[u, v] += H_FD
    Im = c["I"].copy(); Im[u, v] -= H_FD
    return (_D(Ip, c["W"], c["sigma"], c["R"]) - _D(Im, c["W"], c["sigma"], c["R"])) / (2 * H_FD)


def _init(I, W, sigma, R):
    _CASE.update(I=I, W=W, sigma=sigma, R=R)


def fd_case(i, procs):
    case = S.config5_cases(indices=[i])[0]
    I = case.weights
    W = case.w0
    sigma, R = case.sigma, case.R
    A = O.density_map(I, sigma, R)
    D0 = O.lattice_divergence(I, (A,), W, sigma)
    gw = np.zeros((NW, 2))
    for k in range(NW):
        for a in range(2):
            Wp, Wm = W.copy(), W.copy()
            Wp[k, a] += H_FD; Wm[k, a] -= H_FD
            gw[k, a] = (O.lattice_divergence(I, (A,), Wp, sigma) - O.lattice_divergence(I, (A,), Wm, sigma)) / (2 * H_FD)
    coords = [(u, v) for u in range(*CROP) for v in range(*CROP)]
    with mp.Pool(procs, initializer=_init, initargs=(I, W, sigma, R)) as pool:
        gI = np.array(pool.map(_pixel, coords, chunksize=16)).reshape(CROP[1] - CROP[0], -1)
    return {"image": i, "sigma": sigma, "R": R, "M": int(W.shape[0]), "h": H_FD, "crop": list(CROP),
            "D": D0, "grad_weights_crop": gI.tolist(), "grad_w_first": gw.tolist()}


if __name__ == "__main__":
    procs = min(8, os.cpu_count() or 1)
    out = {"what": "central finite differences (h = 1e-4) of the FP64 oracle's lattice divergence",
           "cases": [fd_case(i, procs) for i in (0, 1)]}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fd_config5.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path)

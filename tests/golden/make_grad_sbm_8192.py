"""Writes grad_sbm_8192.npz: the FP64 oracle's loss and gradients for the
differentiation workload (weighted SBM, n = 8192, 32 blocks of 256, mean
degree 24, weights U[0.5, 2], layout U[-20, 20]^2, T = 100 pushes).

Calls only the oracle (and the seeded input generators).  The stored values
are the chain rule through Eq. eq:loss, Eq. eq:pprdist, Definition
def:pprdist and the walk of Section 3.1, evaluated in FP64 by
``oracle.grad_weights``; the GPU parity test compares every edge and
coordinate gradient with them.  A digest of the inputs is stored beside the
values so that the test can tell when the generators no longer produce the
same graph.

Pairs whose 1 - ln z lies within KINK_BAND of a clamp bound of Eq.
eq:pprdist sit on a kink of the loss, where an FP32 evaluation of z may take
either side; the stored gradient takes the clamped side (dDelta/dz = 0) for
them, and their list is stored so that the GPU test can take the same side.

Usage: python tests/golden/make_grad_sbm_8192.py   (about 25 minutes on 8 cores)
"""
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import synth  # noqa: E402

N = 8192
T = 100
ALPHA = 0.15
# FP32 z carries a relative error of a few 1e-7 after T pushes, i.e. the same
# absolute error in 1 - ln z; the band is ten times wider than that.
KINK_BAND = 1e-5


def inputs():
    g = synth.sbm(synth.equal_blocks(N, 32), 0.0753, 6.05e-4, synth.BASE_SEED + 3,
                  weighted=(0.5, 2.0, synth.BASE_SEED + 4))
    X = synth.uniform_layout(N, synth.BASE_SEED + 5) * 20
    return g, X


def digest(g, X):
    h = hashlib.sha256()
    for a in (g.eu.astype(np.int64), g.ev.astype(np.int64), g.weight.astype(np.float32), X.astype(np.float32)):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def main():
    t0 = time.time()
    g, X = inputs()
    print(f"n={g.n} edges={g.m_und} nnz={g.nnz}", flush=True)
    ref = O.grad_weights(N, g.eu, g.ev, g.weight.astype(np.float64), X.astype(np.float64), ALPHA, T,
                         kink_band=KINK_BAND)
    print(f"pairs within {KINK_BAND:g} of a clamp kink: {ref['kink_pairs'].tolist()}", flush=True)
    out = os.path.join(HERE, "grad_sbm_8192.npz")
    np.savez_compressed(out, grad_w=ref["grad_w"], grad_x=ref["grad_x"], loss=np.float64(ref["loss"]),
                        kink_pairs=ref["kink_pairs"].astype(np.int64), kink_band=np.float64(KINK_BAND),
                        digest=np.array(digest(g, X)), n=np.int64(N), T=np.int64(T), alpha=np.float64(ALPHA))
    print(f"wrote {out} in {time.time() - t0:.0f} s: loss={ref['loss']:.12e} "
          f"|grad_w|max={np.abs(ref['grad_w']).max():.4e} |grad_x|max={np.abs(ref['grad_x']).max():.4e}",
          flush=True)


if __name__ == "__main__":
    main()

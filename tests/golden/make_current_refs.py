"""Write the oracle references of the physical-current GPU test (tests/golden/*.npz).

Calls only ``oracle/`` and ``synthetic/``; run on the CPU:

    python tests/golden/make_current_refs.py

The 3x4^3 current workload (``synthetic.workload(6)``: smooth links, mass -1,
mu = 0.3) needs the dense overlap operator with the Schur sign (n = 2304) and the
Daleckii-Krein derivative over all links, about a minute and a half on the host;
the GPU test reads what this script stored:
* ``j_exact``: Tr(D_ov^{-1} dD_ov/dTheta) for every link (complex (4, V));
* ``j_est``: the Z2-noise estimator over the workload's 4 sources with the same
  exact operators (complex (4, V));
* ``x``, ``x_adj``: D_ov^{-1} b and D_ov^{-dag} b for b = the first source.
"""
from __future__ import annotations

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import current as CU  # noqa: E402
from synthetic import workload  # noqa: E402


def main():
    wl = workload(6)
    U, xis = wl.links(), wl.psi()
    D = CU.overlap_dense(U, wl.dims, wl.mass, wl.mu)
    b = xis[0].ravel()
    x = np.linalg.solve(D, b).reshape(xis[0].shape)
    x_adj = np.linalg.solve(D.conj().T, b).reshape(xis[0].shape)
    j_exact = CU.physical_current(U, wl.dims, wl.mass, wl.mu)
    j_est = CU.physical_current(U, wl.dims, wl.mass, wl.mu, xis)
    out = os.path.join(HERE, "physical_current_3x4x4x4.npz")
    np.savez_compressed(out, j_exact=j_exact, j_est=j_est, x=x, x_adj=x_adj)
    print("wrote", out)


if __name__ == "__main__":
    main()

"""Write the stored oracle snapshot used by the full-size parity windows.

Runs the FP64 CPU oracle (and nothing else) on the 1024 x 1024 channel terrain as
configured (dry start, trapezoid inflow hydrograph on the west edge) from t = 0 to
t = 3600 s and stores the nine coefficient planes of every cell that holds water
(sparse: flat cell indices and their values, FP64) with the time and step count.
About 14,000 steps; roughly half an hour on 8 cores.

    python tests/golden/make_snapshots.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import Oracle  # noqa: E402
from paper_2107_02750_amd import scenarios as S  # noqa: E402

OUT = os.path.join(HERE, "fbm_channel_1024_t3600.npz")


def main():
    sc = S.fbm_channel(n=1024)
    o = Oracle(sc)
    t0 = time.time()
    for t in np.arange(300.0, 3600.0 + 1.0, 300.0):
        o.run(float(t))
        s = o.scalars()
        print(f"t={s['t']:.0f} s step {s['step']} ({time.time() - t0:.0f} s)", flush=True)
    planes = o.planes().reshape(9, -1)
    idx = np.nonzero(np.any(planes != 0.0, axis=0))[0].astype(np.int64)
    s = o.scalars()
    np.savez_compressed(OUT, idx=idx, vals=planes[:, idx], nx=sc.nx, ny=sc.ny, t=s["t"],
                        step=s["step"], mass=s["mass"], mass_in=s["mass_in"],
                        mass_out=s["mass_out"], mass_clip=s["mass_clip"])
    print(f"wrote {OUT}: {idx.size} cells", flush=True)


if __name__ == "__main__":
    main()

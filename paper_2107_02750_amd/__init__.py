"""MI355X-native uniform-grid DG2 shallow-water step (arXiv:2107.02750, Sect. 2.1.1).

The GPU library (`csrc/`, built into `libdg2.so`) exposes a C interface declared in
`include/dg2.h`; `dg2.py` is its thin ctypes binding. Import the binding explicitly
(`from paper_2107_02750_amd import dg2`) so that importing the package stays cheap.
"""

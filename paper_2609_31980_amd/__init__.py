"""Exact fixed-radius nearest-neighbour search on AMD Instinct MI355X.

The search runs in libfrnn.so (hand-written HIP for gfx950) behind the C ABI
of include/frnn.h; `paper_2609_31980_amd.frnn` is its Python binding and
`paper_2609_31980_amd.inputs` holds the seeded synthetic workloads.
"""

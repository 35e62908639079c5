"""FP64 CPU oracle of the hybrid thermal pseudo-potential LB step (Hu & Liu, arXiv:1812.10375).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may import this package.  The GPU library never imports it and the
two share no code; what they share is the seeded input generator in
``paper_1812_10375_amd.scenarios``, which holds none of the method's arithmetic.
"""
from .build import build_oracle, library_path  # noqa: F401

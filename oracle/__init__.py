"""Plain FP64 CPU oracle for the AWRTRD / SAWRTRD core-update sweep.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import it.  It shares no code with the HIP
library (``paper_2305_09044_amd``) and imports nothing from it; the two meet only
through the seeded inputs of ``synth``.

Modules: ``tr`` (TR format, Def. 1-2, Thm. 1), ``awrtrd`` (eqs. 7-18, Alg. 1),
``rng`` (sketch index sampling).  Parity unpinned: the 'quantile' kernel-width rule
(own rule; the paper's adaptive rule is not given in its text).
"""
from . import awrtrd, rng, tr  # noqa: F401

"""FP64 CPU oracle of the PCA-based, incrementally pruned, data-driven distance
comparison inside an IVF search.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this
package.  The GPU library (``paper_2404_16322_amd``) never imports, links or
calls it, and shares no code with it: the only common dependency is the seeded
input generator module ``synthdata``, which contains none of the method's
arithmetic.
"""
from .ddc_oracle import *  # noqa: F401,F403

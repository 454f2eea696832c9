"""MI355X-native continuous relaxations for dense CRFs (Desmaison et al.,
ECCV 2016): permutohedral-lattice pairwise filter, Frank-Wolfe QP, CCCP DC
and LP subgradient, as HIP kernels for gfx950 behind a C ABI.

``paper_1608_06192_amd.dcrf`` is the binding of ``libdcrf.so``;
``paper_1608_06192_amd.synth`` holds the seeded synthetic inputs.
"""

__all__ = ["dcrf", "synth"]

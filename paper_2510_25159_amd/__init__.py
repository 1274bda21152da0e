"""MI355X-native batched generalized-winding-number containment queries on
trimmed surfaces (Bao, Shen, Wang: fast and robust point containment queries
on trimmed surfaces).  The compute path lives in ``csrc/`` (HIP for gfx950)
behind the C ABI declared in ``include/wn.h``; ``wn`` is its Python binding.
"""

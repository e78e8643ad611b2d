"""MI355X-native generalized BB/FG permanent (arXiv:2309.07027).

The compute path is the C-ABI library ``libbbfg.so`` (hand-written HIP for
gfx950); :mod:`paper_2309_07027_amd.binding` is its thin ctypes binding.
Importing the package itself loads nothing, so the input generators in
:mod:`paper_2309_07027_amd.inputs` can be used without a GPU.
"""
__all__ = ["inputs", "binding"]

"""MI355X-native FAS multigrid solve of the constrained-ADM constraint and gauge
equations (Barrera-Hinojosa & Li 2019, sec. 4).

The compute path is the HIP library ``libgrmg.so`` (C ABI, see include/gr.h);
``paper_1905_08890_amd.grmg`` is its ctypes binding.  Nothing is imported
eagerly so that the input generators stay importable without a GPU.
"""
__all__ = ["grmg", "synth"]

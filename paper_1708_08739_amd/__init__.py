"""MI355X-native RV(r)-pruned betweenness of one vertex (arxiv 1708.08739).

The compute path is the C-ABI library ``libbcd.so`` (HIP kernels for gfx950);
``paper_1708_08739_amd.bcd`` is its ctypes binding.  ``graphgen`` draws the
seeded synthetic inputs.  Importing the package loads nothing native.
"""

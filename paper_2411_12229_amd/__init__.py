"""MI355X (gfx950) query path of SymphonyQG (arXiv 2411.12229).

``paper_2411_12229_amd.qg`` binds the C ABI of ``libqg.so`` (include/qg.h):
the HIP kernels that rotate queries on the matrix cores, encode RaBitQ blocks
and run Algorithm 1 over a quantization-graph index resident in HBM.
``paper_2411_12229_amd.build`` compiles the library.
"""

"""MI355X-native evaluator for multi-objective dual simplex-mesh deformable
image registration: objectives, partial evaluations and fold checks of a whole
population of coupled tetrahedral-mesh transformations, computed by HIP kernels
for gfx950 behind a C ABI (``include/dsm.h``).

``paper_2202_11001_amd.dsm`` is the binding of the shared library;
``paper_2202_11001_amd.workloads`` draws seeded synthetic inputs.
"""

"""MI355X-native (gfx950) Vlasov-Poisson library: the fourth-order
finite-volume Vlasov right-hand side, velocity-moment reduction, periodic
Poisson solve, field injection and RK4 stepping of Hittinger & Banks,
"Block-Structured Adaptive Mesh Refinement Algorithms for Vlasov
Simulation", as hand-written HIP kernels behind the C ABI in include/vp.h.

The binding lives in `paper_1204_3853_amd.vp`; importing the package does
not load the HIP library.
"""

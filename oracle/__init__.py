"""Plain FP64 CPU oracle for the even-odd Wilson-Dirac hot path of HiRep v2
(arXiv:2503.06721).

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) may import, call, link or execute anything in this package.
Its only users are the test-suite, the smoke check and the CPU-baseline leg
of the benchmark.

Every function is a direct, slow, obviously-correct transcription of the
definition it cites (NumPy complex128; no spin projection, no even-odd
index tricks, no fusion), so that it can be checked against the paper by
eye.  It shares no code with the GPU path; both only consume the seeded
inputs built by ``paper_2503_06721_amd.synth``.

Modules
-------
lattice     geometry, parity, half-field maps, shifts with boundary phases
gamma       Pauli matrices, e_mu, gamma_mu (chiral basis), gamma_5
reps        SU(N) generators, FUND/ADJ/SYM/2AS maps U -> U_R, T^a_R, T_R, C_2
dirac       hopping term, D_m, even-odd blocks, D-hat, source prep/reconstruct
cg          textbook conjugate gradient on D-hat^dagger D-hat
force       pseudofermion action and its link derivative
reductions  FastTwoSum, Neumaier, second-order Neumaier, double-double sums
dense       dense matrices of the operators for brute-force checks
"""

"""MI355X-native rotating IMEX-DG hot path (HIP kernels behind a C-ABI library).

The compiled library is loaded on first use of `paper_2605_29598_amd.binding`;
importing this package loads nothing.
"""

"""Single-seed Lanczos-CG for Hermitian positive definite systems with many
right-hand sides, on AMD Instinct MI355X (gfx950).

The HIP library (``csrc/``, C ABI declared in ``include/seedcg.h``) is loaded
lazily by :mod:`paper_0810_0330_amd.api`; importing this package does not
touch the GPU.
"""
__all__ = ["api", "synth"]

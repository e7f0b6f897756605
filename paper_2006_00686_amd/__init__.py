"""MI355X-native discrete X-ray transform (pixel/voxel basis) and its adjoint.

The compute path is the C-ABI library libxrt.so (hand-written gfx950 HIP kernels);
Python only marshals arguments.  Importing this package does not load the library:
`paper_2006_00686_amd.xrt` does, and fails loudly when it is missing.
"""
__all__ = ["inputs"]

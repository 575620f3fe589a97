"""Import of the HIP library for test modules.

Where a GPU is present the import must succeed: a missing or broken
libdls.so fails the tests loudly instead of skipping them.  Without a GPU
(CPU-only runs, which deselect the GPU tests) a missing library skips the
module."""
import pytest


def load():
    try:
        import paper_1709_02599_amd as dls
        return dls
    except ImportError:
        try:
            import torch
            gpu = torch.cuda.is_available()
        except ImportError:
            gpu = False
        if gpu:
            raise
        pytest.skip("paper_1709_02599_amd is not built", allow_module_level=True)

"""MI355X-native checkpointed adjoint FWI gradient with lossily compressed
checkpoints (Kukreja et al., "Lossy Checkpoint Compression in Full Waveform
Inversion").  The compute path is libfwigrad.so (HIP, gfx950) behind the C
ABI of include/fwigrad.h; ``fwigrad`` is its ctypes binding and ``autograd``
the torch.autograd.Function over it.
"""
from . import fwigrad  # noqa: F401

__all__ = ["fwigrad"]

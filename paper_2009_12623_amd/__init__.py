"""MI355X-native checkpointed adjoint FWI gradient with lossily compressed
checkpoints (Kukreja et al., "Lossy Checkpoint Compression in Full Waveform
Inversion").  The compute path is libfwigrad.so (HIP, gfx950) behind the C
ABI of include/fwigrad.h.  Modules: ``fwigrad`` (its ctypes binding, with
the torch.autograd.Function ops ``FwiFunction`` / ``FwiBatchFunction`` and
``FwiOperator``), ``costmodel`` (schedule counts, unit costs, slot and
tolerance choice), ``fwi`` (the gradient-descent loop), ``studies`` and
``metrics`` (the paper's experiments and error measures), ``build`` (hipcc
build of the library).
"""
from . import fwigrad  # noqa: F401

__all__ = ["fwigrad"]

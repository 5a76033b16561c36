"""MI355X-native stepper for networks of multi-compartment cells.

The hot path (mechanisms, implicit-Euler assembly, Hines solve, threshold
detection, event delivery, spike exchange, adjoint) runs in the HIP library
libarbmi.so behind the C ABI of include/arbmi.h; `arbmi` is its binding and
`grad` the torch.autograd wrapper of the adjoint.
"""
from . import arbmi  # noqa: F401

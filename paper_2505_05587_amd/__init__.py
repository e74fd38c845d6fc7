"""SteepGS hot path on AMD Instinct MI355X (gfx950).

The HIP library ``libsteepgs.so`` (C ABI in ``include/steepgs.h``) holds every
stage: projection, instance sort, forward blend, backward with splitting
matrices, Steepest Density Control.  ``_lib`` is its ctypes binding,
``pipeline`` the buffer orchestration, ``step`` the batched graph-captured
step and ``autograd`` the ``torch.autograd.Function`` wrapper.  ``scenes``
draws seeded synthetic inputs.
"""
__all__ = ["scenes"]

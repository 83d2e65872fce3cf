"""MI355X-native stochastic Galerkin solver with the hierarchical Schur complement preconditioner.

The compute path is the HIP library ``libsgpc.so`` (C interface in
``include/sg.h``); ``binding`` marshals torch device tensors into it and
``autograd`` wraps the adjoint gradient as a ``torch.autograd.Function``.
Importing ``binding`` fails if the library has not been built.
"""

__all__ = ["binding", "autograd"]


def __getattr__(name):
    if name in ("binding", "autograd"):
        import importlib
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)

"""MI355X (gfx950) implementation of the ghost-gluon Dyson-Schwinger solver of
Hopfer, Alkofer and Haase (arXiv:1206.1779): residual, Newton matrix and
Newton solve as hand-written HIP kernels behind a C ABI (``include/dse.h``).

``paper_1206_1779_amd.dse`` is the thin Python binding (argument marshalling
only; every step runs in the HIP library, which must be built first with
``python -m paper_1206_1779_amd.build``)."""

__all__ = ["dse", "build"]

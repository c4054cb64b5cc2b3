"""Batched forward dynamics of serial chains on MI355X (gfx950), after Yang,
Wu and Pan (arXiv 1609.06779): JSIIA, ABIA and CFA built from a parallel scan
(block bi-diagonal systems) and odd-even elimination (block tri-diagonal
systems), hand-written in HIP behind the C-ABI of include/fd.h.

``synth`` (seeded inputs) imports without the GPU library; ``Model``,
``scan6`` and ``btd_solve6`` load libfd.so on first use and raise if it has
not been built.
"""

__all__ = ["Model", "scan6", "btd_solve6", "forward_dynamics", "rollout"]


def __getattr__(name):
    if name in ("Model", "scan6", "btd_solve6", "forward_dynamics", "rollout"):
        from . import fd
        return getattr(fd, name)
    raise AttributeError(name)

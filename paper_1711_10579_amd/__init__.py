"""MI355X-native Newton power flow (arXiv:1711.10579, Sec. II-III).

The compute path is the HIP library built from ``csrc/`` for gfx950; the C
ABI is declared in ``include/pf.h`` and bound in ``binding`` (loaded lazily so
that ``build`` can run before the library exists).
"""

__all__ = ["binding", "build"]


def __getattr__(name):
    if name == "binding":
        import importlib

        return importlib.import_module(__name__ + ".binding")
    raise AttributeError(name)

"""MI355X-native retrieval of the closest pre-simulated tumours (arXiv 2205.04550).

The GPU library is ``libtumordb.so`` (C ABI in ``include/tumordb.h``); this
package binds it with ctypes and uses torch only for device memory and
streams. The binding is imported on first use, so that ``build`` can run
before the library exists.
"""
_EXPORTS = ("DB_KMAX", "DbError", "TumorDB", "storage_bytes")


def __getattr__(name):
    if name in _EXPORTS:
        from . import binding
        return getattr(binding, name)
    raise AttributeError(name)

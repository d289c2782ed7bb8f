"""MI355X-native batched integrator for a Paul-trapped ion colliding with a cold atom.

The computation lives in libiat.so (HIP kernels for gfx950 behind a C ABI, see include/iat.h);
this package only marshals arguments and uses torch for device memory and streams."""
from ._abi import LibraryMissing, IatError, load as load_library  # noqa: F401
from . import _abi as abi  # noqa: F401


def __getattr__(name):
    # the torch-based front end is imported lazily so that `import paper_2509_15117_amd`
    # stays cheap for the host-only checks
    if name in ("integrate", "integrate_workload", "alloc_obs", "api"):
        import importlib
        api = importlib.import_module(__name__ + ".api")
        return api if name == "api" else getattr(api, name)
    raise AttributeError(name)

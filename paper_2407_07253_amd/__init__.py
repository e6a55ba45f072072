"""MI355X (gfx950) implementation of Vanka-star patch relaxation inside monolithic
phMG V-cycles preconditioning FGMRES, for Taylor-Hood and Scott-Vogelius Stokes
discretisations.

* ``frontend``  -- host-side problem set-up (assembly, patches, transfers) that
  produces the inputs of the C ABI;
* ``_lib``      -- ctypes binding of ``libphmg.so`` (HIP kernels + host runtime);
* ``build``     -- compiles ``libphmg.so`` for gfx950.

``Hierarchy`` (from ``_lib``) is imported lazily so that the front-end can be
used on machines where the library has not been built yet.
"""


def __getattr__(name):
    if name in ("Hierarchy", "PhmgError", "last_error"):
        from . import _lib
        return getattr(_lib, name)
    raise AttributeError(name)

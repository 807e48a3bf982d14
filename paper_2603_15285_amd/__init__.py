"""MI355X (gfx950) implementation of the rotational-alignment path of Matcha
(frequency-marched Newton refinement of a band-limited SO(3) correlation).

Submodules: ``matcha`` (binding of libmatcha.so, imported on demand because it needs
torch and the built HIP library) and ``synth`` (seeded synthetic inputs)."""
from . import synth  # noqa: F401

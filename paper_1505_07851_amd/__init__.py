"""MI355X (gfx950) C-PCM / ISWIG solvation path of arXiv:1505.07851.

Every computation runs in libpcm.so (hand-written HIP behind the C ABI of include/pcm.h);
this package only marshals arguments.  Importing it without the built library fails.
"""
from ._lib import lib as _load_lib

_load_lib()

from .api import (Batch, Context, Graph, Molecule, PCMError, ThresholdPolicy, dynamic_threshold,  # noqa: E402
                  octree_partition, rbj_partition)
from .autograd import PCMEnergy, pcm_energy  # noqa: E402

__all__ = ["Batch", "Context", "Graph", "Molecule", "PCMError", "PCMEnergy", "ThresholdPolicy", "dynamic_threshold",
           "octree_partition", "pcm_energy", "rbj_partition"]

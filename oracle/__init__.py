"""CPU oracle for the acquisition hot path.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check in __graft_entry__ and
the CPU-baseline leg of bench.py may import or execute anything in this
package.  The GPU path (paper_2005_10445_amd) never imports it, and the two
share no code: no kernels, headers, tables, constants or pre/post-processing.

Everything here is FP64 and written from the definitions (see reference.py
for the passages followed and the readings taken where the paper is silent;
learned.py holds the proposal stage: STFT power map, CNN, loss, optimiser and
the proposal-to-segment mapping; fsk.py the FSK searching pipeline: int16
conversion, mixing, composed filters, demodulation, replica, correlation and
peak sums).
"""
from .reference import *  # noqa: F401,F403
from .reference import __all__  # noqa: F401
from . import fsk  # noqa: F401,E402  (FSK searching pipeline, Section 3 steps 1-8)

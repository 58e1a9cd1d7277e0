"""FP64 CPU oracle for PPR / DPPR / PDist / stress layout and their gradients,
and for level-l DPPR by Group Forward-Push.

TEST INFRASTRUCTURE: imported only by tests/, __graft_entry__.smoke() and the
CPU-baseline leg of bench.py.  The HIP library never imports or calls it.
"""
from .pprviz_oracle import *  # noqa: F401,F403
from .gfp_oracle import *  # noqa: F401,F403

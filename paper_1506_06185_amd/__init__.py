"""MI355X (gfx950) HHG multigrid with fault recovery.

Importing the package is cheap; ``paper_1506_06185_amd.hhgr`` loads the HIP
library ``libhhgr.so`` (built by ``paper_1506_06185_amd/build.py``) on first use
and raises if it is missing.  ``paper_1506_06185_amd.inputs`` holds the seeded
synthetic inputs.
"""

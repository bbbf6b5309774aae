"""dmx: batched differentiable soft-contact rigid-body rollouts on MI355X (gfx950).

The compute path is the HIP library ``libdmx.so`` behind the C ABI in
``include/dmx.h``; ``paper_2506_14186_amd.dmx`` is its thin ctypes binding.
"""

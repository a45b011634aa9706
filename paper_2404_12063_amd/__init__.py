"""MI355X (gfx950) FastVPINNs training hot path: HIP kernels behind a C ABI (include/vpinn.h).

Import the binding explicitly (``from paper_2404_12063_amd import vpinn``); importing the
package itself loads nothing.
"""

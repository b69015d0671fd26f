"""MI355X (gfx950) per-box PIC step with in-situ device-side cost assessment
for dynamic load balancing.  The C ABI lives in include/picbal.h; the Python
binding is ``paper_2104_11385_amd.picbal``."""

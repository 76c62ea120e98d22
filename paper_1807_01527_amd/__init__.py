"""MI355X (gfx950) asynchronous-timestamp super-point estimation.

`binding` wraps the HIP library's C ABI (include/at.h); `traffic` produces
seeded synthetic pair streams.  Importing the package loads nothing: the HIP
library is loaded on first use and its absence is an error, not a fallback.
"""

__all__ = ["binding", "traffic"]

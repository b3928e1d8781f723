"""Seeded synthetic string workloads for the Huskysort hot path.

This module only draws data: it holds none of the method's arithmetic (no
coding, no ordering).  Both the CPU oracle (test infrastructure) and the HIP
path consume what it produces.  Every array it returns is a plain numpy array:

* ``elems``   -- uint8 (ASCII or byte strings, one byte per element) or uint16
                 (UTF-16 strings, one code unit per character), all strings
                 packed back to back;
* ``offsets`` -- uint64[n + 1], element offsets, ``offsets[0] == 0``, string i
                 is ``elems[offsets[i]:offsets[i + 1]]``;
* ``seg_offsets`` (batched workloads only) -- uint64[S + 1] string offsets of
                 the independent sort instances.
"""

from .gen import (  # noqa: F401
    StringBatch,
    from_strings,
    config1,
    config2,
    config3,
    config4,
    config5,
    adversarial,
    adversarial_bytes,
    utf8_words,
    ADVERSARIAL_FAMILIES,
    BYTES_FAMILIES,
    CONFIG_SIZES,
)

"""CPU oracle for the octagonal-star screen.

TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the CPU
baseline leg of the benchmark are the only callers.  The product package
never imports this package, and this package never imports the product
package: the two share no code.  Inputs come from the separate ``synth``
package, which holds no screening arithmetic.

``oracle.core`` wraps a plain C implementation (``oss_oracle.c``) that sums
every star pixel by pixel and compares features cross-multiplied in 128-bit
integers.  ``oracle.enum_star`` is an independent pure-Python enumerator of
the star's pixel sets, used on tiny inputs to pin the C code.
"""
from .core import (  # noqa: F401
    build,
    threads,
    square_half,
    star_weight,
    star_area,
    gradient,
    star_features,
    template_features,
    feature_pass,
    screen_positions,
    screen_full,
    mask_and_list,
    F_SUM,
    F_SQ,
    F_GRAD,
)

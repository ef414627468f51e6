"""MI355X-native lookback ray marching (the hot path of arXiv 2609.09322's method).

The package is a thin binding over ``libdart.so``; see ``include/dart.h`` for the
C ABI and ``dart.py`` for the Python names (identical to the C entry points).
"""
from .dart import *  # noqa: F401,F403
from .dart import DartError, Server, Stack, View  # noqa: F401

"""MI355X-native CCZ4 FD4 hot path (arXiv:2406.11626): C-ABI HIP library + ctypes binding."""
from . import ccz4  # noqa: F401

from .circuits import *  # noqa: F401,F403
from .circuits import Gate, pack  # noqa: F401
from . import noise  # noqa: F401

"""``python -m paper_2603_07850_amd [OPTIONS] LIMIT``: the command-line verifier."""
import sys

from .cli import main

sys.exit(main())
